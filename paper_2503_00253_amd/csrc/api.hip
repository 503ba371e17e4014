// Host runtime of the InFo-ESRF library: argument validation, workspace
// planning, stream ordering of the kernels, and the C entry points of
// include/infoesrf.h.
//
// Update pipeline (Sec. 3.2 and Appendix E):
//   1. mu, Z from the forecast ensemble (eq. 2.9); b_i = R^{-1/2} H z_i.
//   2. Ritz pairs of S by a randomized eigendecomposition (the preconditioner).
//   3. For every system s = (q, i): solve (1 + s_q) u + S u = b_i by PCG with the
//      limited-memory preconditioner, inside an iterative-refinement loop whose
//      residuals are always formed in FP64 (the inner applies may be FP32/BF16).
//   4. u_bar_i = sum_q p_q u_{q,i};  z_a^(i) = z^(i) - P H^T R^{-1/2} u_bar_i.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstddef>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>
#include <type_traits>
#include <vector>

#include "internal.hpp"
#include "net.hpp"

namespace infoesrf {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

namespace {

inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Bump allocator over the caller's workspace; a null base only measures.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    off = (size_t)round_up((int64_t)off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    return p;
  }
};

constexpr int kChunk = 128;  // rows per reduction chunk

// ------------------------------------------------------------------ kernels local to the runtime
// The call's flags and H's column counts start at zero.
__global__ void k_input_zero(int32_t* flags, int32_t* fallbacks, int32_t* col_cnt, int64_t n) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) col_cnt[t] = 0;
  if (t == 0) {
    *flags = 0;
    *fallbacks = 0;
  }
}

// The element checks of the inputs in one pass: X finite (else the numeric flag); r_var positive
// and finite, and, when declared, each observation one point of the stated lattice (else the
// bad-input flag; h_idx[k] is read only when rows 0..k hold one entry each).
__global__ void k_input_checks(const double* X, int64_t nN, const double* r_var, int64_t m, int lattice,
                               const int32_t* h_ptr, const int32_t* h_idx, infoesrf_lattice lat, int32_t nx,
                               int32_t* flags) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < nN && !isfinite(X[t])) atomicOr(flags, kFlagNumeric);
  if (t < m) {
    bool bad = !(r_var[t] > 0.0 && isfinite(r_var[t]));
    if (lattice) {
      const int64_t a = t / lat.nxo, b = t % lat.nxo;
      const int64_t want = (int64_t)(lat.z0 + a * lat.sz) * nx + (lat.x0 + b * lat.sx);
      bad = bad || h_ptr[t] != (int32_t)t || h_ptr[t + 1] != (int32_t)(t + 1) || h_idx[t] != want;
    }
    if (bad) atomicOr(flags, kFlagBadInput);
  }
}

// Observation columns scattered to the state grid, R^{-1/2} weighted, when H is the declared
// sub-lattice (row k = a nxo + b holds its one entry, index k, at state point
// (z0 + a sz, x0 + b sx)): V[c][j] = w_k / sqrt(r_var_k) P[act_c][k] at the observed points, zero
// elsewhere; the transposed-H scatter's sums, each of one term.
__global__ void k_scatter_lattice(const double* __restrict__ P, int64_t ldp, const int32_t* __restrict__ act,
                                  const int32_t* __restrict__ nact, infoesrf_lattice lat, int32_t nx,
                                  const double* __restrict__ h_w, const double* __restrict__ r_var, int64_t n,
                                  int64_t m, int64_t Bmax, double* __restrict__ V, int64_t ldv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * Bmax) return;
  const int64_t c = t / n, j = t % n;
  const int32_t na = nact ? *nact : (int32_t)Bmax;
  double acc = 0.0;
  if (c < na) {
    const int64_t dz = j / nx - lat.z0, dx = j % nx - lat.x0;
    if (dz >= 0 && dx >= 0 && dz % lat.sz == 0 && dx % lat.sx == 0) {
      const int64_t a = dz / lat.sz, b = dx / lat.sx;
      const int64_t k = a * lat.nxo + b;
      if (a < lat.nzo && b < lat.nxo && k < m) acc = h_w[k] / sqrt(r_var[k]) * P[(int64_t)act[c] * ldp + k];
    }
  }
  V[c * ldv + j] = acc;
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) b[t] = a[t];
}

__global__ void k_widen(const float* __restrict__ a, double* __restrict__ b, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) b[t] = (double)a[t];
}

// out[c * ldo + r] = in[c * ldi + r] converted (r < rows); rows <= r < ldo are zeroed when pad != 0
// and left untouched otherwise (the caller's padding)
template <typename Tin, typename Tout>
__global__ void k_convert_cols(const Tin* __restrict__ in, int64_t ldi, int64_t rows, int64_t cols,
                               Tout* __restrict__ out, int64_t ldo, int pad) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ldo * cols) return;
  const int64_t c = t / ldo, r = t % ldo;
  if (r >= rows && !pad) return;
  const float zero = 0.f;
  if constexpr (std::is_same<Tout, __hip_bfloat16>::value)
    out[t] = __float2bfloat16(r < rows ? (float)in[c * ldi + r] : zero);
  else
    out[t] = (Tout)(r < rows ? in[c * ldi + r] : (Tin)0);
}

// column-major FP64 (ld) -> system-major BF16 (ldk >= n, zero padded)
__global__ void k_to_bf16_cols(const double* __restrict__ V, int64_t ldv, int64_t n, int64_t ldk, int64_t B,
                               __hip_bfloat16* __restrict__ out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ldk * B) return;
  const int64_t k = t % ldk, b = t / ldk;
  out[t] = __float2bfloat16(k < n ? (float)V[k + b * ldv] : 0.f);
}

// Set per-system shifts: sigma[q*N + i] = s_q; the values arrive by kernel argument (capture safe).
struct Nodes {
  double s[kMaxQ];
  double p[kMaxQ];
};
// Shifts past the Q N + extra systems, up to spad, are zero.
__global__ void k_set_nodes(Nodes nd, int32_t Q, int64_t N, double* sigma, double* pw, int64_t extra,
                            double extra_sigma, int64_t spad) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < (int64_t)Q * N) sigma[t] = nd.s[t / N];
  if (t < Q) pw[t] = nd.p[t];
  if (t < extra) sigma[(int64_t)Q * N + t] = extra_sigma;
  if (t >= (int64_t)Q * N + extra && t < spad) sigma[t] = 0.0;
}

// The per-system counters of a solve start at zero: iterations, sweeps, final status; and the
// apply-count adjustment.
__global__ void k_zero_counters(int32_t* __restrict__ iters, int32_t* __restrict__ sweeps,
                                int32_t* __restrict__ fdone, int64_t count, int64_t* __restrict__ app_adj) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) {
    iters[i] = 0;
    sweeps[i] = 0;
    fdone[i] = 0;
  }
  if (i == 0) *app_adj = 0;
}

// Sweep bookkeeping from true residual norms (iterative refinement).
//   fdone: 1 converged (rn <= rtol bn), 2 failed (iteration cap or non-finite), 0 needs work.
//   done (inner PCG status) = fdone ? 1 : 0; thresh = absolute inner target.
// The trunk's inputs of the members (see infoesrf.h): X[i * m + r] = sqrt(m) b_i[r] / ||b_i||, with
// member i's right-hand side in system i (node 0) of the system-major b (ld).
__global__ void k_member_features(const double* __restrict__ b, int64_t ld, const double* __restrict__ bn, int64_t m,
                                  int64_t N, float* __restrict__ X) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N * m) return;
  const int64_t i = t / m, r = t % m;
  const double nb = bn[i];
  X[t] = nb > 0.0 ? (float)(sqrt((double)m) * b[i * ld + r] / nb) : 0.f;
}

// The shift head: system s = q N + i starts from u_s = (||b_s|| / sqrt(m)) sum_d c^(d+1) Y_i[d],
// c = 1 / (1 + sigma_s), Y (N x D x m) the trunk's outputs; a system whose start is not finite
// starts from zero and is counted in *fallbacks.  One block per system.
__global__ __launch_bounds__(256) void k_head_init(const float* __restrict__ Y, int D, int64_t m, int64_t N,
                                                   const double* __restrict__ sigma, const double* __restrict__ bn,
                                                   double* __restrict__ u, int64_t ld, int32_t* __restrict__ fallbacks) {
  __shared__ int bad;
  const int64_t s = blockIdx.x, i = s % N;
  const double c = 1.0 / (1.0 + sigma[s]);
  const float* y = Y + i * D * m;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const double sc = bn[s] / sqrt((double)m);
  for (int64_t r = threadIdx.x; r < m; r += 256) {
    double v = 0.0, p = c;
    for (int d = 0; d < D; ++d) {
      v += p * (double)y[d * m + r];
      p *= c;
    }
    if (!isfinite(v)) bad = 1;
    u[s * ld + r] = sc * v;
  }
  __syncthreads();
  if (bad) {
    for (int64_t r = threadIdx.x; r < m; r += 256) u[s * ld + r] = 0.0;
    if (threadIdx.x == 0) atomicAdd(fallbacks, 1);
  }
}

// Training pairs of the Q N systems s = q N + i: cq[q] = 1 / (1 + sigma_{q N}) and
// T[(i Q + q) m + r] = sqrt(m) u_s[r] / ||b_s|| (FP32).
__global__ void k_net_targets(const double* __restrict__ u, int64_t ld, const double* __restrict__ bn,
                              const double* __restrict__ sigma, int64_t m, int64_t N, int Q, float* __restrict__ cq,
                              float* __restrict__ T) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < Q) cq[t] = (float)(1.0 / (1.0 + sigma[t * N]));
  if (t >= (int64_t)Q * N * m) return;
  const int64_t r = t % m, iq = t / m, i = iq / Q, q = iq % Q, s = q * N + i;
  const double nb = bn[s];
  T[t] = nb > 0.0 ? (float)(sqrt((double)m) * u[s * ld + r] / nb) : 0.f;
}

//   With a fixed iteration count, reaching it sets fdone = 3 (finished, not a failure) and the
//   inner target is 0, so the inner PCG stops only at the count or on an exactly zero residual.
// The sweep status of system s from its residual norm r and right-hand-side norm b.
__device__ inline void sweep_status_one(int64_t s, double b, double r, double rtol, double inner_rtol, int fp64_inner,
                                        const int32_t* iters, int max_iter, int fixed, double* relres,
                                        int32_t* fdone, int32_t* done, double* thresh, int32_t* sweeps,
                                        int count_sweep, int32_t* flags) {
  if (fdone[s] != 0) {
    done[s] = 1;
    return;
  }
  if (count_sweep) sweeps[s] += 1;
  const double rr = b > 0.0 ? r / b : 0.0;
  relres[s] = rr;
  if (!isfinite(rr)) {
    atomicOr(flags, kFlagNumeric);
    fdone[s] = 2;
    done[s] = 1;
    return;
  }
  if (rr <= rtol) {
    fdone[s] = 1;
    done[s] = 1;
    return;
  }
  if (iters[s] >= max_iter) {
    fdone[s] = fixed ? 3 : 2;
    done[s] = 1;
    return;
  }
  done[s] = 0;
  const double target = 0.5 * rtol * b;
  thresh[s] = fixed ? 0.0 : (fp64_inner ? target : fmax(inner_rtol * r, target));
}

__global__ void k_sweep_status(const double* rn, const double* bn, double rtol, double inner_rtol, int fp64_inner,
                               const int32_t* iters, int max_iter, int fixed, double* relres, int32_t* fdone,
                               int32_t* done, double* thresh, int32_t* sweeps, int count_sweep, int64_t S,
                               int32_t* flags) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  sweep_status_one(s, bn[s], rn[s], rtol, inner_rtol, fp64_inner, iters, max_iter, fixed, relres, fdone, done, thresh,
                   sweeps, count_sweep, flags);
}

// The start of a zero-start solve, one 256-thread block per system slot s < spad: the counters
// zeroed (and the apply-count correction); for s < S the norm of b, u = 0 and the first sweep's
// status (its residual is b itself).
__global__ __launch_bounds__(256) void k_solve_start(const double* __restrict__ b, int64_t m, int64_t ld, int64_t S,
                                                     double* __restrict__ bnorm, double* __restrict__ u,
                                                     int32_t* iters, int32_t* sweeps, int32_t* fdone,
                                                     int64_t* app_adj, double rtol, double inner_rtol, int fp64_inner,
                                                     int max_iter, int fixed, double* relres, int32_t* done,
                                                     double* thresh, int32_t* flags) {
  __shared__ double part[4];
  const int64_t s = blockIdx.x;
  const int t = threadIdx.x;
  if (t == 0) {
    iters[s] = 0;
    sweeps[s] = 0;
    fdone[s] = 0;
    if (s == 0) *app_adj = 0;
  }
  if (s >= S) return;
  double acc = 0.0;
  for (int64_t r = t; r < ld; r += 256) {
    if (r < m) {
      const double x = b[s * ld + r];
      acc += x * x;
    }
    u[s * ld + r] = 0.0;
  }
  const double w = wave_sum_dpp(acc);
  if ((t & 63) == 63) part[t >> 6] = w;
  __syncthreads();
  if (t == 0) {
    const double bn = sqrt(((part[0] + part[1]) + part[2]) + part[3]);
    bnorm[s] = bn;
    sweep_status_one(s, bn, bn, rtol, inner_rtol, fp64_inner, iters, max_iter, fixed, relres, fdone, done, thresh,
                     sweeps, 0, flags);
  }
}

// Counters of the call (deterministic reduction over systems in one block).
// Applies saved by a multi-shift process: every member iteration is one apply, while the
// per-system counts add one per live shift.  adj = sum_i mit[i] - sum_s iters[s] (one block).
__global__ void k_msc_adjust(const int32_t* iters, int64_t S, const int32_t* mit, int64_t N, int64_t* adj) {
  __shared__ int64_t acc[256];
  const int t = threadIdx.x;
  int64_t a = 0;
  for (int64_t i = t; i < N; i += 256) a += mit[i];
  for (int64_t s = t; s < S; s += 256) a -= iters[s];
  acc[t] = a;
  __syncthreads();
  if (t == 0) {
    int64_t tot = 0;
    for (int j = 0; j < 256; ++j) tot += acc[j];
    *adj = tot;
  }
}

// Also, when given: the live count (done == 0) into *nact_out, a copy of the counters into out2,
// and the per-system statistics (iterations, relative residuals, converged at tol).
__global__ void k_finish_counters(const int32_t* iters, const int32_t* sweeps, const int32_t* fdone, int64_t S,
                                  int64_t extra_fp64_applies, const int64_t* adj, int inner_fp64, int fixed,
                                  const int32_t* flags, const int32_t* fallbacks, int64_t* out, const int32_t* done,
                                  int32_t* nact_out, int64_t* out2, const double* relres, int32_t* oi, double* orr,
                                  uint8_t* oc, double tol, int64_t* mirror) {
  // 1024 threads: up to 1024 systems in one pass of loads
  constexpr int NT = 1024, NW = NT / 64;
  __shared__ int64_t acc[5][NW];
  const int t = threadIdx.x;
  // the single words thread 0 reports, loaded before the per-system pass (not after it)
  int32_t f = 0, fb = 0;
  int64_t ad = 0;
  if (t == 0) {
    f = *flags;
    fb = fallbacks ? *fallbacks : 0;
    ad = adj ? *adj : 0;
  }
  int64_t it = 0, sw = 0, nc = 0, mx = 0, lv = 0;
  for (int64_t s = t; s < S; s += NT) {
    it += iters[s];
    sw += sweeps[s];
    nc += (fdone[s] != 1);
    mx = max(mx, (int64_t)iters[s]);
    if (done) lv += (done[s] == 0);
    if (oi) oi[s] = iters[s];
    if (orr) orr[s] = relres[s];
    if (oc) oc[s] = (done[s] == 1 && relres[s] <= tol) ? 1 : 0;
  }
  // wavefront sums by shuffles, then the wavefronts in order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    it += __shfl_xor(it, o, 64);
    sw += __shfl_xor(sw, o, 64);
    nc += __shfl_xor(nc, o, 64);
    mx = max(mx, __shfl_xor(mx, o, 64));
    lv += __shfl_xor(lv, o, 64);
  }
  if ((t & 63) == 0) {
    acc[0][t >> 6] = it;
    acc[1][t >> 6] = sw;
    acc[2][t >> 6] = nc;
    acc[3][t >> 6] = mx;
    acc[4][t >> 6] = lv;
  }
  __syncthreads();
  if (t == 0) {
    int64_t a = 0, b = 0, c = 0, d = 0, live = 0;
    for (int j = 0; j < NW; ++j) {
      live += acc[4][j];
      a += acc[0][j];
      b += acc[1][j];
      c += acc[2][j];
      d = max(d, acc[3][j]);
    }
    out[INFOESRF_CNT_ITERATIONS] = a;
    out[INFOESRF_CNT_SWEEPS] = b;
    out[INFOESRF_CNT_NOT_CONVERGED] = c;
    out[INFOESRF_CNT_MAX_ITERS] = d;
    const int64_t ai = a + ad;  // inner applies
    out[INFOESRF_CNT_APPLIES] = ai + b + extra_fp64_applies;
    out[INFOESRF_CNT_APPLIES_FP64] = (inner_fp64 ? ai : 0) + b + extra_fp64_applies;
    out[INFOESRF_CNT_FALLBACKS] = fb;
    int64_t status = INFOESRF_OK;
    if (f & kFlagBadInput) status = INFOESRF_ERR_INVALID_ARG;
    else if (f & kFlagNumeric) status = INFOESRF_ERR_NUMERIC;
    else if (f & kFlagNotSPD) status = INFOESRF_ERR_NOT_SPD;
    else if (c > 0 && !fixed) status = INFOESRF_WARN_NOT_CONVERGED;  // a fixed count is what was asked
    out[INFOESRF_CNT_STATUS] = status;
    if (out2)
      for (int j = 0; j < INFOESRF_NUM_COUNTERS; ++j) out2[j] = out[j];
    if (nact_out) *nact_out = (int32_t)live;
    if (mirror) {  // the live count in the low word of the first entry, then the counters
      mirror[0] = (int64_t)(uint32_t)live;
      for (int j = 0; j < INFOESRF_NUM_COUNTERS; ++j) mirror[1 + j] = out[j];
    }
  }
}

inline unsigned nb(int64_t c) { return (unsigned)((c + 255) / 256); }

// ------------------------------------------------------------------ plan

struct Options {
  double rtol, inner_rtol;
  int fixed;  // > 0: run exactly this many PCG iterations per system
  int max_iter, p, k;  // Ritz pairs, sketch columns
  Prec inner;
  int solver;
  int host_sync;
  int rows_per_wave;
  bool obs;
  infoesrf_lattice lat;
  uint64_t seed;
  const double* sketch;
  int warm;
  const void* net;
  bool band;  // covariance applies through the explicit band of P
  int sform;  // INFOESRF_S_*: requested form of S
  int msc_q0 = -1;  // multi-shift perturbation solve: the base node (-1: not used)
  int bcg_Q = 0;    // block perturbation solve: number of nodes (0: not used)
  int tail = 64;    // live systems at which one persistent launch finishes the PCG loop (-1: never)
  int warm_fp32 = 0;  // learned start: FP32 inference instead of BF16 on MFMA
};

struct Inst {
  const infoesrf_problem* P = nullptr;
  int64_t n = 0, N = 0, m = 0;
  bool dense = false, obs = false;
  infoesrf_lattice lat{};  // the declared observation lattice (obs)
  // S assembled as a dense m x m matrix (column-major, ld = lds; FP32 copy for FP32 inner applies)
  bool sd = false;
  double* Sd = nullptr;
  float* Sd32 = nullptr;
  int64_t lds = 0;
  // the PCG vectors and their applies live in observation space (lattice domain or dense S)
  bool odom() const { return obs || sd; }
  Grid gs{};  // state grid
  Grid go{};  // observation lattice grid (obs domain)
  double *mu = nullptr, *Z = nullptr, *Zt = nullptr, *subtab = nullptr;
  float *Z32 = nullptr, *Zt32 = nullptr, *tab32 = nullptr, *subtab32 = nullptr;
  int32_t *col_cnt = nullptr, *col_ptr = nullptr, *row_of = nullptr;
  double* w_of = nullptr;
  double *diagS = nullptr, *dmin = nullptr;
  int32_t* flags = nullptr;
  int32_t* fallbacks = nullptr;
  int64_t* counters = nullptr;
  // explicit bands of P (band form): state grid, and observed lattice (obs domain); FP64 and,
  // for MIXED_FP32 inner applies in that domain, an FP32 copy
  bool band = false;
  void *bandS = nullptr, *bandS32 = nullptr, *bandO = nullptr, *bandO32 = nullptr;
  // FP32 copies of the observed-lattice band and of the dense S in the persistent kernel's packed
  // layout (four stencil entries of a row in 16 bytes), for FP32 inner applies
  float *bandQ32 = nullptr, *SdQ32 = nullptr;
  // on a declared lattice with the band form: the final apply's rectangular band (state points x
  // the lattice points of their window) in place of the state grid's band
  bool rect = false;
  RectGeom rg{};
  double* rectS = nullptr;
  // learned warm start: network buffers for the members (inputs, trunk outputs, the network's
  // own workspace)
  const Net* net = nullptr;
  bool warm_fp32 = false;  // FP32 inference instead of BF16 on MFMA
  int64_t wmem = 0;        // members the trunk runs on
  float *wX = nullptr, *wY = nullptr;
  void* wnet = nullptr;
  size_t wnet_bytes = 0;
};

// Solver state: observation-space vectors are system-major, system s at s * ldm.
struct Sys {
  int64_t S = 0, ldm = 0, Spad = 0;
  double *b = nullptr, *u = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
  double *bnorm = nullptr, *rn = nullptr, *rz = nullptr, *relres = nullptr, *rel_in = nullptr, *sigma = nullptr,
         *thresh = nullptr, *pw = nullptr;
  int32_t *iters = nullptr, *sweeps = nullptr, *done = nullptr, *fdone = nullptr;
  int32_t *act = nullptr, *nact = nullptr, *act2 = nullptr, *nact2 = nullptr;
  // the last host check's words in the pinned stage's layout: the live count, then the counters
  int64_t* stage = nullptr;
  // multi-shift CG (SOLVER_MULTISHIFT): per-system zeta pair, per-member base scalars
  double *zeta = nullptr, *zeta_prev = nullptr, *mrr = nullptr, *malpha = nullptr, *mbeta = nullptr;
  int32_t* mit = nullptr;
  int64_t* app_adj = nullptr;  // applies counter correction: member iterations replace system iterations
  int32_t* qctr = nullptr;     // work-queue counter of the persistent finish
  // block PCG (SOLVER_BLOCK): W = C P, partial and reduced products, coefficients, node states
  double *bw = nullptr, *bpart = nullptr, *bred = nullptr, *bcoef = nullptr;
  int32_t* bdone = nullptr;
};

struct Pre {
  int k = 0, p = 0;
  double *Om = nullptr, *Y = nullptr, *Qb = nullptr, *SQ = nullptr, *Tk = nullptr, *evec = nullptr,
         *evals = nullptr, *Rinv = nullptr, *sel = nullptr, *Phi = nullptr, *SPhi = nullptr, *theta = nullptr,
         *G = nullptr, *gscr = nullptr, *sig = nullptr;
  int32_t *act = nullptr, *nact = nullptr;
};

// Apply buffers (input V, output T), system-major with leading dimension round_up(rows, 64).
struct Buf {
  void* V = nullptr;
  void* T = nullptr;
  int64_t cols = 0;  // columns allocated
};

struct Fin {
  double* ubar = nullptr;  // system-major, N (or 1) columns of ldm
  int32_t *act = nullptr, *nact = nullptr;
};

struct Plan {
  Inst in;
  Sys sy;
  Pre pr;
  Buf bf;
  Fin fn;
  size_t bytes = 0;
};

inline int64_t ld64(int64_t rows) { return round_up(rows, 64); }
// Room reserved for the CSC copy of H: 64 entries per row on average, or 16 per state variable
// (wide observation channels), whichever is larger.
inline int64_t nnz_bound(const infoesrf_problem* P) { return std::max<int64_t>(P->m * 64, P->n * 16); }

int check_problem(const infoesrf_problem* P) {
  IE_CHECK(P != nullptr, INFOESRF_ERR_INVALID_ARG, "problem is NULL");
  IE_CHECK(P->N >= 2, INFOESRF_ERR_INVALID_ARG, "ensemble size N must be >= 2");
  IE_CHECK(P->m >= 1, INFOESRF_ERR_INVALID_ARG, "observation count m must be >= 1");
  IE_CHECK(P->n >= 1, INFOESRF_ERR_INVALID_ARG, "state dimension n must be >= 1");
  IE_CHECK(P->n < (1LL << 30) && P->N < (1LL << 20), INFOESRF_ERR_INVALID_ARG, "dimensions too large");
  IE_CHECK(P->m <= 4096, INFOESRF_ERR_INVALID_ARG, "m must be <= 4096 (one workgroup holds a system's vectors)");
  IE_CHECK(P->X && P->h_ptr && P->h_idx && P->h_w && P->r_var, INFOESRF_ERR_INVALID_ARG,
           "X, h_ptr, h_idx, h_w and r_var must be non-NULL");
  const infoesrf_loc& L = P->loc;
  if (L.kind == INFOESRF_LOC_DENSE) {
    IE_CHECK(L.dense != nullptr, INFOESRF_ERR_INVALID_ARG, "dense localization pointer is NULL");
    IE_CHECK(P->n <= 8192, INFOESRF_ERR_INVALID_ARG, "dense localization limited to n <= 8192");
    return 0;
  }
  IE_CHECK(L.kind == INFOESRF_LOC_STENCIL, INFOESRF_ERR_INVALID_ARG, "unknown localization kind");
  IE_CHECK(L.table != nullptr, INFOESRF_ERR_INVALID_ARG, "stencil table is NULL");
  IE_CHECK(L.nz >= 1 && L.nx >= 1 && (int64_t)L.nz * L.nx == P->n, INFOESRF_ERR_INVALID_ARG,
           "stencil grid nz*nx must equal n");
  IE_CHECK(L.bz >= 0 && L.bx >= 0, INFOESRF_ERR_INVALID_ARG, "stencil half-extents must be >= 0");
  IE_CHECK(!L.periodic_x || L.nx >= 2 * L.bx + 1, INFOESRF_ERR_INVALID_ARG, "periodic x needs nx >= 2bx+1");
  IE_CHECK(!L.periodic_z || L.nz >= 2 * L.bz + 1, INFOESRF_ERR_INVALID_ARG, "periodic z needs nz >= 2bz+1");
  IE_CHECK((int64_t)(2 * L.bz + 1) * (2 * L.bx + 41) * 8 <= 64 * 1024, INFOESRF_ERR_INVALID_ARG,
           "stencil too large for one workgroup LDS: (2bz+1)(2bx+41)*8 must be <= 64 KiB");
  return 0;
}

int resolve_options(const infoesrf_problem* P, const infoesrf_opts* o, Options& op) {
  infoesrf_opts d;
  infoesrf_default_opts(&d);
  if (!o) o = &d;
  IE_CHECK(o->rtol > 0.0 && o->rtol < 1.0, INFOESRF_ERR_INVALID_ARG, "rtol must be in (0, 1)");
  IE_CHECK(o->max_iter >= 1, INFOESRF_ERR_INVALID_ARG, "max_iter must be >= 1");
  IE_CHECK(o->fixed_iters >= 0, INFOESRF_ERR_INVALID_ARG, "fixed_iters must be >= 0");
  IE_CHECK(o->tail_systems >= -1, INFOESRF_ERR_INVALID_ARG, "tail_systems must be >= -1");
  IE_CHECK(o->fixed_iters == 0 || o->precision == INFOESRF_FP64, INFOESRF_ERR_INVALID_ARG,
           "fixed_iters needs precision FP64 (a mixed solve counts inner and outer iterations)");
  IE_CHECK(o->n_ritz >= 0 && o->oversample >= 0, INFOESRF_ERR_INVALID_ARG, "n_ritz, oversample must be >= 0");
  const int p = o->n_ritz;
  IE_CHECK(p == 0 || p == 4 || p == 8 || p == 10 || p == 12 || p == 16 || p == 20, INFOESRF_ERR_INVALID_ARG,
           "n_ritz must be one of 0, 4, 8, 10, 12, 16, 20");
  IE_CHECK(p + o->oversample <= kMaxSketch, INFOESRF_ERR_INVALID_ARG, "n_ritz + oversample must be <= 48");
  IE_CHECK(p == 0 || p + o->oversample <= P->m, INFOESRF_ERR_INVALID_ARG, "n_ritz + oversample must be <= m");
  IE_CHECK(o->precision >= INFOESRF_FP64 && o->precision <= INFOESRF_MIXED_BF16, INFOESRF_ERR_INVALID_ARG,
           "unknown precision");
  IE_CHECK(o->solver != INFOESRF_SOLVER_MULTISHIFT ||
               (o->precision == INFOESRF_FP64 && o->warm_start == INFOESRF_START_ZERO),
           INFOESRF_ERR_INVALID_ARG, "the multi-shift solver needs precision FP64 and the zero start");
  IE_CHECK(o->solver != INFOESRF_SOLVER_BLOCK ||
               (o->precision == INFOESRF_FP64 && o->warm_start == INFOESRF_START_ZERO && P->N <= 64),
           INFOESRF_ERR_INVALID_ARG, "the block solver needs precision FP64, the zero start and N <= 64");
  IE_CHECK(o->solver >= INFOESRF_SOLVER_PLAIN && o->solver <= INFOESRF_SOLVER_BLOCK, INFOESRF_ERR_INVALID_ARG,
           "unknown solver");
  IE_CHECK(o->warm_start == INFOESRF_START_ZERO || o->warm_start == INFOESRF_START_LEARNED, INFOESRF_ERR_INVALID_ARG,
           "unknown warm_start");
  IE_CHECK(o->warm_start != INFOESRF_START_LEARNED || o->net != nullptr, INFOESRF_ERR_INVALID_ARG,
           "the learned warm start needs opts->net");
  IE_CHECK(o->apply_domain == INFOESRF_DOMAIN_STATE || o->apply_domain == INFOESRF_DOMAIN_OBS_LATTICE,
           INFOESRF_ERR_INVALID_ARG, "unknown apply domain");
  IE_CHECK(o->tile_rows == 0 || o->tile_rows == 16 || o->tile_rows == 32 || o->tile_rows == 64 ||
               o->tile_rows == 128,
           INFOESRF_ERR_INVALID_ARG, "tile_rows must be 0, 16, 32, 64 or 128");
  IE_CHECK(o->cov_form >= INFOESRF_COV_AUTO && o->cov_form <= INFOESRF_COV_BAND, INFOESRF_ERR_INVALID_ARG,
           "unknown cov_form");
  IE_CHECK(o->s_form >= INFOESRF_S_AUTO && o->s_form <= INFOESRF_S_DENSE, INFOESRF_ERR_INVALID_ARG,
           "unknown s_form");
  IE_CHECK(o->s_form != INFOESRF_S_DENSE || (o->precision != INFOESRF_MIXED_BF16 && P->m <= kDenseSMax),
           INFOESRF_ERR_INVALID_ARG, "the dense form of S needs FP64 or MIXED_FP32 and m <= 16384");
  {
    const bool stencil = P->loc.kind == INFOESRF_LOC_STENCIL;
    const bool prec_ok = o->precision != INFOESRF_MIXED_BF16;
    IE_CHECK(o->cov_form != INFOESRF_COV_BAND || (stencil && prec_ok), INFOESRF_ERR_INVALID_ARG,
             "the band form needs a stencil localization and FP64 or MIXED_FP32");
    const double planes = stencil ? (double)(2 * P->loc.bz + 1) * (2 * P->loc.bx + 1) : 0.0;
    const double bytes = planes * (double)round_up(P->n, 64) * 12.0;  // FP64 + FP32 copies, state grid
    op.band = o->cov_form == INFOESRF_COV_BAND ||
              (o->cov_form == INFOESRF_COV_AUTO && stencil && prec_ok && bytes <= 2.0 * (1ull << 30));
  }
  op.rtol = o->rtol;
  op.sform = o->s_form;
  op.tail = o->tail_systems == 0 ? INT32_MAX : o->tail_systems;
  op.warm_fp32 = o->warm_fp32 != 0;
  op.fixed = o->fixed_iters;
  op.max_iter = op.fixed > 0 ? op.fixed : o->max_iter;
  op.p = p;
  op.k = p > 0 ? p + o->oversample : 0;
  op.inner = (o->precision == INFOESRF_FP64) ? Prec::F64 : (o->precision == INFOESRF_MIXED_FP32 ? Prec::F32 : Prec::BF16);
  // FP32 inner applies: a first sweep taken to 1e-7 of the residual lets many systems pass the
  // FP64 check at once and shortens the longest solves (n = 4096 lattice: 18015 -> 17729
  // iterations, 79 -> 78 at most, 1280 -> 1163 sweeps); looser targets restart more, and
  // tighter ones iterate on a recursive residual the FP32 apply no longer tracks
  op.inner_rtol = o->inner_rtol > 0.0 ? o->inner_rtol : (op.inner == Prec::F32 ? 1e-7 : 1e-2);
  op.solver = o->solver;
  op.host_sync = o->host_sync;
  op.rows_per_wave = o->tile_rows;  // 0: chosen per launch from the batch size
  op.obs = (o->apply_domain == INFOESRF_DOMAIN_OBS_LATTICE);
  op.lat = o->lattice;
  op.seed = o->seed;
  op.sketch = o->sketch;
  op.warm = o->warm_start;
  op.net = o->net;
  if (op.obs) {
    const infoesrf_loc& L = P->loc;
    const infoesrf_lattice& a = op.lat;
    IE_CHECK(L.kind == INFOESRF_LOC_STENCIL, INFOESRF_ERR_INVALID_ARG, "lattice domain needs a stencil localization");
    IE_CHECK(a.sz >= 1 && a.sx >= 1 && a.nzo >= 1 && a.nxo >= 1 && a.z0 >= 0 && a.x0 >= 0,
             INFOESRF_ERR_INVALID_ARG, "bad lattice description");
    IE_CHECK((int64_t)a.nzo * a.nxo == P->m, INFOESRF_ERR_INVALID_ARG, "lattice nzo*nxo must equal m");
    IE_CHECK(a.z0 + (int64_t)(a.nzo - 1) * a.sz < L.nz && a.x0 + (int64_t)(a.nxo - 1) * a.sx < L.nx,
             INFOESRF_ERR_INVALID_ARG, "lattice leaves the grid");
    IE_CHECK(!L.periodic_x || (int64_t)a.nxo * a.sx == L.nx, INFOESRF_ERR_INVALID_ARG,
             "periodic x lattice must cover the axis (nxo*sx == nx)");
    IE_CHECK(!L.periodic_z || (int64_t)a.nzo * a.sz == L.nz, INFOESRF_ERR_INVALID_ARG,
             "periodic z lattice must cover the axis (nzo*sz == nz)");
  }
  return 0;
}

// Whether S is assembled as a dense m x m matrix for a call with S systems (INFOESRF_S_AUTO:
// when a product with it costs at most half of an apply of P in the working domain, counted as
// rows x stencil points for the band, times N for the operator form, and the m applies that
// form it are few next to the applies of the solves).
bool use_dense_s(const infoesrf_problem* P, const Options& op, int64_t S) {
  if (op.sform == INFOESRF_S_DENSE) return true;
  if (op.sform == INFOESRF_S_OPERATOR || op.inner == Prec::BF16) return false;
  const int64_t m = P->m;
  if (m > kDenseSAuto) return false;
  double rows, points;
  if (P->loc.kind == INFOESRF_LOC_STENCIL) {
    const infoesrf_loc& L = P->loc;
    if (op.obs) {
      rows = (double)m;
      points = (double)(2 * (L.bz / op.lat.sz) + 1) * (2 * (L.bx / op.lat.sx) + 1);
    } else {
      rows = (double)P->n;
      points = (double)(2 * L.bz + 1) * (2 * L.bx + 1);
    }
  } else {
    rows = (double)P->n;
    points = (double)P->n;
  }
  const double per_vector = rows * points * (op.band ? 1.0 : (double)P->N);
  return 2.0 * (double)m * (double)m <= per_vector && m <= 8 * (S + op.k + 16);
}

// Lay out every buffer of one call.  `S` systems, `nfin` final state-space columns.
void plan_layout(Plan& pl, Arena& ar, const infoesrf_problem* P, const Options& op, int64_t S, int64_t nfin) {
  Inst& in = pl.in;
  in.P = P;
  in.n = P->n;
  in.N = P->N;
  in.m = P->m;
  in.dense = (P->loc.kind == INFOESRF_LOC_DENSE);
  in.obs = op.obs;
  in.lat = op.lat;
  in.band = op.band;
  in.sd = use_dense_s(P, op, S);
  // the operator form in a low precision needs FP32 copies of Z and the stencil (with a dense S
  // every low-precision apply is a product with the FP32 copy of S)
  const bool low = (op.inner != Prec::F64) && !op.band && !in.sd;
  in.mu = ar.take<double>(in.n);
  in.Z = ar.take<double>(in.n * in.N);
  in.Z32 = (low && !in.obs) ? ar.take<float>(in.n * in.N) : nullptr;
  if (!in.dense) {
    const infoesrf_loc& L = P->loc;
    in.gs = Grid{L.nz, L.nx, L.periodic_z, L.periodic_x, L.bz, L.bx, L.table, nullptr, nullptr};
    if (low) in.tab32 = ar.take<float>((2 * L.bz + 1) * (2 * L.bx + 1));
    in.gs.table32 = in.tab32;
  }
  if (in.obs) {
    const infoesrf_loc& L = P->loc;
    const infoesrf_lattice& a = op.lat;
    const int bzs = L.bz / a.sz, bxs = L.bx / a.sx;
    in.Zt = ar.take<double>(in.m * in.N);
    in.Zt32 = low ? ar.take<float>(in.m * in.N) : nullptr;
    in.subtab = ar.take<double>((2 * bzs + 1) * (2 * bxs + 1));
    in.subtab32 = low ? ar.take<float>((2 * bzs + 1) * (2 * bxs + 1)) : nullptr;
    const int pz = L.periodic_z && (int64_t)a.nzo * a.sz == L.nz;
    const int px = L.periodic_x && (int64_t)a.nxo * a.sx == L.nx;
    in.go = Grid{a.nzo, a.nxo, pz, px, bzs, bxs, in.subtab, in.subtab32, nullptr};
  }
  if (in.band) {
    const infoesrf_loc& L = P->loc;
    const bool f32 = op.inner == Prec::F32;
    const int64_t ps = (int64_t)(2 * L.bz + 1) * (2 * L.bx + 1) * ld64(in.n);
    in.rect = in.obs && !in.dense && rect_fits(in.gs, op.lat, in.N);
    if (in.rect) {
      in.rg = rect_geom(in.gs, op.lat);
      in.rectS = ar.take<double>((int64_t)in.rg.wz * in.rg.wx * ld64(in.n));
    }
    in.bandS = in.rect ? nullptr : ar.take<double>(ps);
    in.bandS32 = (f32 && !in.obs && !in.sd) ? ar.take<float>(ps) : nullptr;
    if (in.obs) {
      const int64_t po = (int64_t)(2 * in.go.bz + 1) * (2 * in.go.bx + 1) * ld64(in.m);
      in.bandO = ar.take<double>(po);
      in.bandO32 = (f32 && !in.sd) ? ar.take<float>(po) : nullptr;
      in.bandQ32 = (f32 && !in.sd)
                       ? ar.take<float>((int64_t)(2 * in.go.bz + 1) * ((2 * in.go.bx + 1 + 3) / 4) * ld64(in.m) * 4)
                       : nullptr;
    }
  }
  if (in.sd) {
    in.lds = ld64(in.m);
    in.Sd = ar.take<double>(in.lds * in.m);
    in.Sd32 = (op.inner == Prec::F32) ? ar.take<float>(in.lds * in.m) : nullptr;
    in.SdQ32 = (op.inner == Prec::F32) ? ar.take<float>((in.m + 3) / 4 * in.lds * 4) : nullptr;
  }
  in.col_cnt = ar.take<int32_t>(in.n);
  in.col_ptr = ar.take<int32_t>(in.n + 1);
  in.diagS = ar.take<double>(in.m);
  in.dmin = ar.take<double>(1);
  in.flags = ar.take<int32_t>(1);
  in.fallbacks = ar.take<int32_t>(1);
  in.counters = ar.take<int64_t>(INFOESRF_NUM_COUNTERS);
  if (op.warm == INFOESRF_START_LEARNED && S > 1) {
    in.net = static_cast<const Net*>(op.net);
    in.warm_fp32 = op.warm_fp32;
    in.wmem = std::min<int64_t>(S, in.N);
    in.wX = ar.take<float>(in.wmem * in.m);
    in.wY = ar.take<float>(in.wmem * in.net->D * in.m);
    in.wnet_bytes = net_ws_bytes(*in.net, in.wmem, 1, in.m, false);
    in.wnet = ar.take<char>((int64_t)in.wnet_bytes);
  }

  Sys& sy = pl.sy;
  sy.S = S;
  sy.ldm = ld64(in.m);
  sy.Spad = round_up(S, kSysTile);
  const int64_t ms = sy.ldm * sy.Spad;
  sy.b = ar.take<double>(ms);
  sy.u = ar.take<double>(ms);
  sy.x = ar.take<double>(ms);
  sy.r = ar.take<double>(ms);
  sy.p = ar.take<double>(ms);
  sy.q = ar.take<double>(ms);
  sy.bnorm = ar.take<double>(sy.Spad);
  sy.rn = ar.take<double>(sy.Spad);
  sy.rz = ar.take<double>(sy.Spad);
  sy.relres = ar.take<double>(sy.Spad);
  sy.rel_in = ar.take<double>(sy.Spad);
  sy.sigma = ar.take<double>(sy.Spad);
  sy.thresh = ar.take<double>(sy.Spad);
  sy.pw = ar.take<double>(kMaxQ);
  sy.iters = ar.take<int32_t>(sy.Spad);
  sy.sweeps = ar.take<int32_t>(sy.Spad);
  sy.done = ar.take<int32_t>(sy.Spad);
  sy.fdone = ar.take<int32_t>(sy.Spad);
  sy.act = ar.take<int32_t>(sy.Spad);
  sy.nact = ar.take<int32_t>(2);  // list length, live count
  sy.act2 = ar.take<int32_t>(sy.Spad);
  sy.nact2 = ar.take<int32_t>(2);
  sy.stage = ar.take<int64_t>(INFOESRF_NUM_COUNTERS + 1);
  if (op.solver == INFOESRF_SOLVER_MULTISHIFT) {
    const int64_t nm = round_up(std::max<int64_t>(in.N, 1), kSysTile);
    sy.zeta = ar.take<double>(sy.Spad);
    sy.zeta_prev = ar.take<double>(sy.Spad);
    sy.mrr = ar.take<double>(nm);
    sy.malpha = ar.take<double>(nm);
    sy.mbeta = ar.take<double>(nm);
    sy.mit = ar.take<int32_t>(nm);
  }
  sy.app_adj = ar.take<int64_t>(1);
  sy.qctr = ar.take<int32_t>(1);
  if (op.solver == INFOESRF_SOLVER_BLOCK && S > 1 && S % in.N == 0) {
    const int Qb = (int)(S / in.N);
    sy.bw = ar.take<double>(ms);
    sy.bpart = ar.take<double>(bcg_partial_doubles(in.m, in.N, op.p, Qb));
    sy.bred = ar.take<double>(bcg_reduced_doubles(in.N, op.p, Qb));
    sy.bcoef = ar.take<double>(bcg_coef_doubles(in.N, op.p, Qb));
    sy.bdone = ar.take<int32_t>(Qb);
  }

  Pre& pr = pl.pr;
  pr.k = op.k;
  pr.p = op.p;
  if (op.k > 0) {
    const int64_t kl = round_up(op.k, kSysTile);
    pr.Om = ar.take<double>(sy.ldm * kl);
    pr.Y = ar.take<double>(sy.ldm * kl);
    pr.Qb = ar.take<double>(sy.ldm * kl);
    pr.SQ = ar.take<double>(sy.ldm * kl);
    pr.Tk = ar.take<double>(op.k * op.k);
    pr.evec = ar.take<double>(op.k * op.k);
    pr.evals = ar.take<double>(op.k);
    pr.Rinv = ar.take<double>(op.k * op.k);
    pr.sel = ar.take<double>(op.k * op.p);
    pr.Phi = ar.take<double>(sy.ldm * op.p);
    pr.SPhi = ar.take<double>(sy.ldm * op.p);
    pr.theta = ar.take<double>(op.p);
    pr.G = ar.take<double>(3 * op.p * op.p);
    pr.gscr = ar.take<double>((int64_t)gram_chunks(in.m) * op.k * op.k);
    pr.sig = ar.take<double>(kl);
    pr.act = ar.take<int32_t>(kl);
    pr.nact = ar.take<int32_t>(1);
  }
  Fin& fn = pl.fn;
  const int64_t nf = round_up(std::max<int64_t>(nfin, 1), kSysTile);
  fn.ubar = ar.take<double>(sy.ldm * nf);
  fn.act = ar.take<int32_t>(nf);
  fn.nact = ar.take<int32_t>(1);

  // apply buffers: rows x columns in FP64 (enough for every precision)
  const int64_t cols = std::max<int64_t>({sy.Spad, round_up(op.k, kSysTile), nf, 16});
  const int64_t rows = std::max<int64_t>(ld64(in.n), ld64(in.m));
  pl.bf.cols = cols;
  pl.bf.V = ar.take<double>(rows * cols);
  pl.bf.T = ar.take<double>(rows * cols);
}

// ------------------------------------------------------------------ apply
// Tile variant of a covariance launch: the caller's choice, else a rule from the
// measured sweep on MI355X (large batches: 32 rows x 32 systems per block; small
// batches: 16 x 32, which doubles the number of blocks).
TuneKey op_key(int form, Prec p, const Grid& g, int64_t N) {
  return TuneKey{form, (int)p, g.nz, g.nx, g.bz, g.bx, (int)N};
}
int tile_for(int requested, int64_t B, const TuneKey& k) {
  if (requested) return requested;
  const int t = tuned_choice(k, B);  // a measured choice (infoesrf_autotune), if any
  if (t == 16 || t == 32 || t == 64 || t == 128) return t;
  return B >= 128 ? 32 : 16;
}
// BF16 blocks: 16 rows x 128 / 64 / 32 systems by batch size
int tile_for_bf16(int requested, int64_t B, const TuneKey& k) {
  if (requested) return requested;
  const int t = tuned_choice(k, B);
  if (t == 16 || t == 32 || t == 64 || t == 128) return t;
  return B >= 384 ? 128 : (B >= 96 ? 64 : 16);
}

// T = S-part of the apply for the listed columns of Pin (system-major, ldp); when Qout is given,
// Qout[:, s] = (1 + sigma_s) Pin[:, s] + S Pin[:, s] as well.  v_ready: the observation-domain
// apply buffer already holds the listed columns (written by the fused PCG kernel).  zero_counter
// (nullable) is set to 0 on the stream before the apply finishes; the stencil kernels do it
// themselves, which saves a launch per PCG iteration.
// T = P V for the first Bmax (or *nact) columns of the apply buffer V, in the working domain of
// the covariance (observed lattice or state grid) and the form chosen for P.
int apply_raw(Plan& pl, Prec prec, int64_t Bmax, const int32_t* nact, int rows_per_wave, hipStream_t st,
              int32_t* zero_counter) {
  Inst& in = pl.in;
  const int64_t rows = in.obs ? in.m : in.n;
  const int64_t ldr = ld64(rows);
  const Grid& g = in.obs ? in.go : in.gs;
  if (Bmax == 0 || in.dense) {
    if (zero_counter) IE_HIP(launch_fill_i32(zero_counter, 0, 2, st));
    zero_counter = nullptr;
  }
  if (in.band) {
    IE_CHECK(prec != Prec::BF16, INFOESRF_ERR_INVALID_ARG, "the band form has no BF16 apply");
    const void* band = in.obs ? (prec == Prec::F64 ? in.bandO : in.bandO32)
                              : (prec == Prec::F64 ? in.bandS : in.bandS32);
    IE_HIP(cov_band_timed(prec, g, band, ldr, pl.bf.V, ldr, pl.bf.cols, Bmax, nact, pl.bf.T, ldr, st, zero_counter));
  } else if (prec == Prec::BF16) {
    IE_CHECK(!in.dense, INFOESRF_ERR_INVALID_ARG, "dense localization supports FP64 only");
    const float* Zu = in.obs ? in.Zt32 : in.Z32;
    IE_HIP(cov_bf16_timed(g, Zu, rows, in.N, (const __hip_bfloat16*)pl.bf.V, ldr, pl.bf.cols, Bmax, nact,
                          (float*)pl.bf.T, ldr, tile_for_bf16(rows_per_wave, Bmax, op_key(2, prec, g, in.N)), st,
                          zero_counter));
  } else if (in.dense) {
    IE_CHECK(prec == Prec::F64, INFOESRF_ERR_INVALID_ARG, "dense localization supports FP64 only");
    IE_HIP(launch_cov_dense(in.P->loc.dense, in.Z, in.n, in.N, (const double*)pl.bf.V, ldr, Bmax, (double*)pl.bf.T,
                            ldr, st));
  } else {
    const void* Zu = (prec == Prec::F64) ? (in.obs ? (const void*)in.Zt : (const void*)in.Z)
                                         : (in.obs ? (const void*)in.Zt32 : (const void*)in.Z32);
    IE_HIP(cov_stencil_timed(prec, g, Zu, rows, in.N, pl.bf.V, ldr, pl.bf.cols, Bmax, nact, pl.bf.T, ldr,
                             tile_for(rows_per_wave, Bmax, op_key(1, prec, g, in.N)), st, zero_counter));
  }
  return 0;
}

// S = R^{-1/2} H P H^T R^{-1/2} as a dense m x m matrix: P applied to H^T R^{-1/2} e_k (state
// domain) or to e_k on the observed lattice (whose members already carry H and R^{-1/2}), a
// buffer's worth of columns at a time, then symmetrized.
int build_dense_s(Plan& pl, const Options& op, hipStream_t st) {
  Inst& in = pl.in;
  const infoesrf_problem* P = in.P;
  const int64_t rows = in.obs ? in.m : in.n;
  const int64_t ldr = ld64(rows);
  double* V = static_cast<double*>(pl.bf.V);
  for (int64_t j0 = 0; j0 < in.m; j0 += pl.bf.cols) {
    const int64_t bc = std::min<int64_t>(pl.bf.cols, in.m - j0);
    if (in.obs) {
      IE_HIP(launch_unit_cols(rows, j0, bc, V, ldr, st));
    } else {
      IE_HIP(launch_fill_f64(V, 0.0, ldr * bc, st));
      IE_HIP(launch_scatter_unit_obs(P->h_ptr, P->h_idx, P->h_w, P->r_var, in.n, j0, bc, V, ldr, st));
    }
    IE_TRY(apply_raw(pl, Prec::F64, bc, nullptr, op.rows_per_wave, st, nullptr));
    IE_HIP(launch_gather_s_cols(in.obs ? 1 : 0, static_cast<const double*>(pl.bf.T), ldr, P->h_ptr, P->h_idx,
                                P->h_w, P->r_var, in.n, in.m, j0, bc, in.Sd, in.lds, st));
  }
  IE_HIP(launch_symmetrize(in.Sd, in.m, in.lds, in.Sd32, st));
  if (in.SdQ32) IE_HIP(launch_pack_quads(in.Sd, 1, in.m, in.lds, in.m, in.SdQ32, st));
  return 0;
}

// T = S-part of the apply for the listed columns of Pin (system-major, ldp); when Qout is given,
// Qout[:, s] = (1 + sigma_s) Pin[:, s] + S Pin[:, s] as well.  v_ready: the observation-domain
// apply buffer already holds the listed columns (written by the fused PCG kernel).  zero_counter
// (nullable) is set to 0 on the stream before the apply finishes; the covariance kernels do it
// themselves, which saves a launch per PCG iteration.
int apply_S(Plan& pl, Prec prec, const double* Pin, int64_t ldp, const int32_t* act, const int32_t* nact,
            int64_t Bmax, const double* sigma, double* Qout, int rows_per_wave, hipStream_t st,
            bool v_ready = false, int32_t* zero_counter = nullptr) {
  Inst& in = pl.in;
  const int64_t Bpad = round_up(Bmax, kSysTile);
  const bool od = in.odom();
  const int64_t ldr = ld64(od ? in.m : in.n);
  if (od) {
    if (!v_ready) IE_HIP(launch_gather_active(prec, Pin, ldp, act, nact, in.m, Bpad, pl.bf.V, ldr, st));
  } else {
    IE_HIP(launch_scatter_state(prec, Pin, ldp, act, nact, in.col_ptr, in.row_of, in.w_of, in.P->r_var, in.n, in.m,
                                Bpad, pl.bf.V, ldr, st));
  }
  if (in.sd) {
    const void* Sp = (prec == Prec::F64) ? (const void*)in.Sd : (const void*)in.Sd32;
    IE_CHECK(Sp != nullptr, INFOESRF_ERR_INVALID_ARG, "the dense form of S has no copy in this precision");
    IE_HIP(launch_dense_s_apply(prec, Sp, in.lds, in.m, pl.bf.V, ldr, nact, Bpad, pl.bf.T, ldr, zero_counter, st));
  } else {
    IE_TRY(apply_raw(pl, prec, Bpad, nact, rows_per_wave, st, zero_counter));
  }
  if (Qout)
    IE_HIP(launch_apply_finish(prec, od ? 1 : 0, Pin, ldp, pl.bf.T, ldr, act, nact, sigma, in.P->h_ptr,
                               in.P->h_idx, in.P->h_w, in.P->r_var, in.m, in.n, Bpad, Qout, st));
  return 0;
}

// State-space apply of observation-space columns U (system-major, ld):
// T_state = P H^T R^{-1/2} U, returned in pl.bf.T (system-major FP64, leading dimension ld64(n)).
int apply_state(Plan& pl, const double* U, int64_t ld, const int32_t* act, const int32_t* nact, int64_t ncols,
                int rows_per_wave, hipStream_t st) {
  Inst& in = pl.in;
  const int64_t Bpad = round_up(ncols, kSysTile);
  const int64_t ldr = ld64(in.n);
  if (in.rect) {  // the declared lattice with the band form: the rectangular band on the lattice columns
    IE_HIP(launch_rect_apply(in.rg, in.rectS, ldr, U, ld, act, nact, ncols, static_cast<double*>(pl.bf.T), ldr, st));
    return 0;
  }
  if (in.obs) {  // the declared lattice: no transposed H
    hipLaunchKernelGGL(k_scatter_lattice, dim3(nb(in.n * Bpad)), dim3(256), 0, st, U, ld, act, nact, in.lat,
                       in.P->loc.nx, in.P->h_w, in.P->r_var, in.n, in.m, Bpad, (double*)pl.bf.V, ldr);
    IE_HIP(hipGetLastError());
  } else {
    IE_HIP(launch_scatter_state(Prec::F64, U, ld, act, nact, in.col_ptr, in.row_of, in.w_of, in.P->r_var, in.n,
                                in.m, Bpad, pl.bf.V, ldr, st));
  }
  if (in.band) {
    IE_HIP(cov_band_timed(Prec::F64, in.gs, in.bandS, ldr, pl.bf.V, ldr, pl.bf.cols, ncols, nullptr, pl.bf.T, ldr,
                          st));
  } else if (in.dense) {
    IE_HIP(launch_cov_dense(in.P->loc.dense, in.Z, in.n, in.N, (const double*)pl.bf.V, ldr, ncols,
                            (double*)pl.bf.T, ldr, st));
  } else {
    IE_HIP(cov_stencil_timed(Prec::F64, in.gs, in.Z, in.n, in.N, pl.bf.V, ldr, pl.bf.cols, ncols, nullptr, pl.bf.T,
                             ldr, tile_for(rows_per_wave, ncols, op_key(1, Prec::F64, in.gs, in.N)), st));
  }
  return 0;
}

// ------------------------------------------------------------------ stages
// Pinned words the host reads behind an event: the live count, the input-check flags, the
// counters.
struct HostStage {
  int32_t nact;
  int32_t flags;
  int64_t cnt[INFOESRF_NUM_COUNTERS];
};
static_assert(offsetof(HostStage, cnt) == sizeof(int64_t) &&
                  sizeof(HostStage) == sizeof(int64_t) * (INFOESRF_NUM_COUNTERS + 1),
              "the device stage mirrors this layout");
HostStage* host_stage() {
  static thread_local HostStage* h = nullptr;
  if (!h && hipHostMalloc((void**)&h, sizeof(HostStage), hipHostMallocDefault) != hipSuccess) h = nullptr;
  return h;
}
hipEvent_t host_event() {
  static thread_local hipEvent_t e = nullptr;
  if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) e = nullptr;
  return e;
}


bool tail_inplace(const Plan& pl, const Options& op, TailApply& tap);

// Whether a solve with these options hands every system to the persistent kernel from its first
// sweep (the conditions stage_solve tests): then the batched loop's FP32 band is never applied.
bool persistent_only(const Plan& pl, const Options& op) {
  const Inst& in = pl.in;
  TailApply tap{};
  if (op.tail != INT32_MAX || op.solver != INFOESRF_SOLVER_COMPACT || !tail_inplace(pl, op, tap)) return false;
  const double elem = op.inner == Prec::F32 ? 4.0 : 8.0;
  const double bytes = in.sd ? elem * in.m * in.m : elem * in.m * (2 * in.go.bz + 1) * (2 * in.go.bx + 1);
  return bytes <= 1024.0 * 1024;
}

// solve: the plan serves solves (the autotuner's plan times every apply, so it builds every band)
int stage_setup(Plan& pl, const Options& op, hipStream_t st, bool solve = true) {
  Inst& in = pl.in;
  const infoesrf_problem* P = in.P;
  // 1. input checks (they read H only within its own CSR bounds): the flags and column counts
  //    zeroed, the element checks, the CSR check and count of H.  On a declared lattice the
  //    element checks require every row of H to be its one lattice point (a CSR of m entries,
  //    in range: the lattice lies in the grid), and nothing uses H's transpose: no count.
  const int64_t ncnt = in.obs ? 0 : in.n;
  hipLaunchKernelGGL(k_input_zero, dim3(nb(std::max<int64_t>(ncnt, 1))), dim3(256), 0, st, in.flags, in.fallbacks,
                     in.col_cnt, ncnt);
  IE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_input_checks, dim3(nb(std::max<int64_t>(in.n * in.N, in.m))), dim3(256), 0, st, P->X,
                     in.n * in.N, P->r_var, in.m, in.obs ? 1 : 0, P->h_ptr, P->h_idx, op.lat, P->loc.nx, in.flags);
  IE_HIP(hipGetLastError());
  if (!in.obs) IE_HIP(launch_csc_count(P->h_ptr, P->h_idx, in.m, in.n, nnz_bound(P), in.col_cnt, in.flags, st));
  // with host synchronization the input checks are read from pinned memory behind an event
  HostStage* hs = nullptr;
  hipEvent_t ev = nullptr;
  if (op.host_sync) {
    hs = host_stage();
    ev = host_event();
    IE_CHECK(hs && ev, INFOESRF_ERR_HIP, "pinned host staging or event creation failed");
    IE_HIP(hipMemcpyAsync(&hs->flags, in.flags, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    IE_HIP(hipEventRecord(ev, st));
  }
  // the rest of H's transpose (it writes nothing when a check failed) and the ensemble statistics
  // (which read only X) run meanwhile
  // (on the declared lattice the state scatter needs no transposed H)
  if (!in.obs)
    IE_HIP(launch_csc_finish(P->h_ptr, P->h_idx, P->h_w, in.m, in.n, in.col_cnt, in.col_ptr, in.row_of, in.w_of,
                             in.flags, st));
  // FP32 copies of Z and of the stencil exist only for the operator form in a low precision
  // (plan_layout allocates them under the same condition)
  const bool low = (op.inner != Prec::F64) && !in.band && !in.sd;
  IE_HIP(launch_ens_stats(P->X, in.n, in.N, in.mu, in.Z, in.Z32, st));
  if (op.host_sync) {
    IE_HIP(hipEventSynchronize(ev));
    const int32_t f = hs->flags;
    if (f & kFlagBadInput) {
      set_error(
          "invalid observation operator (CSR out of range, unsorted, more than max(64 m, 16 n) entries, or not the "
          "stated lattice) or r_var <= 0");
      return INFOESRF_ERR_INVALID_ARG;
    }
    if (f & kFlagNumeric) {
      set_error("non-finite value in the forecast ensemble");
      return INFOESRF_ERR_NUMERIC;
    }
  }
  // 2. ensemble and observation-space setup (indices are guarded against invalid values, which
  //    can only reach here when host_sync == 0; the flag then sets the call's status)
  IE_HIP(launch_diag_S(P->h_ptr, P->h_idx, P->h_w, P->r_var, in.Z, in.n, in.N, in.m, in.gs,
                       in.dense ? P->loc.dense : nullptr, in.diagS, st));
  IE_HIP(launch_min_reduce(in.diagS, in.m, in.dmin, st));
  if (!in.dense && low) {
    const infoesrf_loc& L = P->loc;
    IE_CHECK(in.tab32 != nullptr, INFOESRF_ERR_HIP, "internal: FP32 stencil copy not allocated");
    IE_HIP(launch_convert_f32(L.table, in.tab32, (int64_t)(2 * L.bz + 1) * (2 * L.bx + 1), st));
  }
  if (in.obs) {
    const infoesrf_loc& L = P->loc;
    SubTable sub;
    sub.table = L.table;
    sub.bz = L.bz;
    sub.bx = L.bx;
    sub.sz = op.lat.sz;
    sub.sx = op.lat.sx;
    sub.bzs = in.go.bz;
    sub.bxs = in.go.bx;
    sub.out = in.subtab;
    IE_HIP(launch_lattice_members(P->h_idx, P->h_w, P->r_var, in.Z, in.n, in.N, in.m, in.Zt, in.Zt32, st, sub));
    if (low) {
      IE_CHECK(in.subtab32 != nullptr, INFOESRF_ERR_HIP, "internal: FP32 lattice stencil not allocated");
      IE_HIP(launch_convert_f32(in.subtab, in.subtab32, (int64_t)(2 * in.go.bz + 1) * (2 * in.go.bx + 1), st));
    }
  }
  // 3. explicit bands of P (band form): one pass over the members each
  if (in.band) {
    if (in.rect) IE_HIP(launch_rect_build(in.rg, in.Z, in.n, in.Zt, in.m, in.N, in.rectS, ld64(in.n), st));
    else IE_HIP(launch_band_build(Prec::F64, in.gs, in.Z, in.n, in.N, in.bandS, ld64(in.n), st));
    if (in.bandS32) IE_HIP(launch_band_build(Prec::F32, in.gs, in.Z, in.n, in.N, in.bandS32, ld64(in.n), st));
    if (in.obs) {
      IE_HIP(launch_band_build(Prec::F64, in.go, in.Zt, in.m, in.N, in.bandO, ld64(in.m), st));
      if (in.bandO32 && !(solve && persistent_only(pl, op)))
        IE_HIP(launch_band_build(Prec::F32, in.go, in.Zt, in.m, in.N, in.bandO32, ld64(in.m), st));
      if (in.bandQ32)
        IE_HIP(launch_pack_quads(static_cast<const double*>(in.bandO), 2 * in.go.bz + 1, 2 * in.go.bx + 1, ld64(in.m),
                                 in.m, in.bandQ32, st));
    }
  }
  // 4. dense S (m applies of P)
  if (in.sd) IE_TRY(build_dense_s(pl, op, st));
  return 0;
}

// Randomized eigendecomposition of S -> Phi, S Phi, theta, Gram matrices (Appendix E).
int stage_precond(Plan& pl, const Options& op, hipStream_t st) {
  Pre& pr = pl.pr;
  if (pr.p == 0) return 0;
  Inst& in = pl.in;
  const int k = pr.k;
  const int64_t ldm = pl.sy.ldm;
  if (small_basis_fits(k, pr.p, in.m) && in.obs && in.band && !in.sd) {
    // On the observed lattice the band apply reads its input block and writes its output block
    // with the leading dimension of the systems: the sketch is written straight into the input
    // block and Qb copied there by the Cholesky-QR kernel, and S Omega, S Qb are read from the
    // output block in place (with (1 + sigma) = 0 the apply's finish would only copy them out).
    double* V = static_cast<double*>(pl.bf.V);
    const double* T = static_cast<const double*>(pl.bf.T);
    const int64_t Bpad = round_up(k, kSysTile);
    if (op.sketch) {
      IE_HIP(launch_copy_cols(op.sketch, in.m, in.m, k, V, ldm, st));
      IE_HIP(launch_iota(pr.act, pr.nact, k, st));
    } else {
      IE_HIP(launch_sketch_setup(op.seed, in.m, k, V, ldm, pr.act, pr.nact, pr.sig, Bpad, st));
    }
    IE_TRY(apply_raw(pl, Prec::F64, Bpad, pr.nact, op.rows_per_wave, st, nullptr));
    IE_HIP(launch_cholqr2_small(T, in.m, k, ldm, pr.Qb, V, in.flags, st));
    IE_TRY(apply_raw(pl, Prec::F64, Bpad, pr.nact, op.rows_per_wave, st, nullptr));
    IE_HIP(launch_ritz_small(pr.Qb, T, in.m, k, pr.p, ldm, pr.theta, pr.Phi, pr.SPhi, pr.G, st));
    return 0;
  }
  // the k sketch columns are applied as systems 0 .. k-1 with (1 + sigma) = 0: pure S
  if (op.sketch) {
    IE_HIP(launch_copy_cols(op.sketch, in.m, in.m, k, pr.Om, ldm, st));
    IE_HIP(launch_iota(pr.act, pr.nact, k, st));
    IE_HIP(launch_fill_f64(pr.sig, -1.0, round_up(k, kSysTile), st));
  } else {
    IE_HIP(launch_sketch_setup(op.seed, in.m, k, pr.Om, ldm, pr.act, pr.nact, pr.sig, round_up(k, kSysTile), st));
  }
  IE_TRY(apply_S(pl, Prec::F64, pr.Om, ldm, pr.act, pr.nact, k, pr.sig, pr.Y, op.rows_per_wave, st));
  if (small_basis_fits(k, pr.p, in.m)) {  // the small dense steps in two launches
    IE_HIP(launch_cholqr2_small(pr.Y, in.m, k, ldm, pr.Qb, nullptr, in.flags, st));
    IE_TRY(apply_S(pl, Prec::F64, pr.Qb, ldm, pr.act, pr.nact, k, pr.sig, pr.SQ, op.rows_per_wave, st));
    IE_HIP(launch_ritz_small(pr.Qb, pr.SQ, in.m, k, pr.p, ldm, pr.theta, pr.Phi, pr.SPhi, pr.G, st));
    return 0;
  }
  // Cholesky-QR twice: Qb = Y R^{-1}
  const Strided Ys{pr.Y, 1, ldm}, Qs{pr.Qb, 1, ldm};
  IE_HIP(launch_gram(Ys, Ys, in.m, k, pr.Rinv, pr.gscr, st));
  IE_HIP(launch_chol_inv(pr.Rinv, k, in.flags, st));
  IE_HIP(launch_right_mult(Ys, in.m, k, pr.Rinv, k, pr.Qb, 1, ldm, st));
  IE_HIP(launch_gram(Qs, Qs, in.m, k, pr.Rinv, pr.gscr, st));
  IE_HIP(launch_chol_inv(pr.Rinv, k, in.flags, st));
  IE_HIP(launch_right_mult(Qs, in.m, k, pr.Rinv, k, pr.Y, 1, ldm, st));
  IE_HIP(launch_copy_cols(pr.Y, ldm, ldm, k, pr.Qb, ldm, st));
  IE_TRY(apply_S(pl, Prec::F64, pr.Qb, ldm, pr.act, pr.nact, k, pr.sig, pr.SQ, op.rows_per_wave, st));
  const Strided SQs{pr.SQ, 1, ldm};
  IE_HIP(launch_gram(Qs, SQs, in.m, k, pr.Tk, pr.gscr, st));
  IE_HIP(launch_sym_eig(pr.Tk, k, pr.evec, pr.evals, st));
  IE_HIP(launch_lmp_finish(pr.evals, pr.evec, k, pr.p, pr.theta, pr.sel, st));
  const int p = pr.p;
  IE_HIP(launch_right_mult(Qs, in.m, k, pr.sel, p, pr.Phi, 1, ldm, st));  // column-major m x p, ld = ldm
  IE_HIP(launch_right_mult(SQs, in.m, k, pr.sel, p, pr.SPhi, 1, ldm, st));
  const Strided Ph{pr.Phi, 1, ldm}, SPh{pr.SPhi, 1, ldm};
  IE_HIP(launch_gram(Ph, Ph, in.m, p, pr.G, pr.gscr, st));
  IE_HIP(launch_gram(Ph, SPh, in.m, p, pr.G + p * p, pr.gscr, st));
  IE_HIP(launch_gram(SPh, SPh, in.m, p, pr.G + 2 * p * p, pr.gscr, st));
  return 0;
}

// Non-blocking convergence poll.  The host copies the device's live-system count into pinned
// memory behind an event every few iterations and reads it once the event has completed, so the
// stream never drains while the host waits.  At most kDepth copies are in flight; when that many
// are pending the host waits for the oldest, which bounds how far launches run ahead of the
// device (iterations enqueued after convergence find an empty list and return at once).
class LivePoll {
 public:
  static constexpr int kDepth = 2;
  ~LivePoll() {
    // copies still in flight target the thread's pinned words: let them land first
    for (int i = 0; i < pending_; ++i) (void)hipEventSynchronize(ev_[(head_ + i) % kDepth]);
    for (auto& e : ev_)
      if (e) (void)hipEventDestroy(e);
  }
  int init() {
    words_ = pinned_words();
    IE_CHECK(words_ != nullptr, INFOESRF_ERR_HIP, "pinned host allocation failed");
    for (auto& e : ev_) IE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return 0;
  }
  // Enqueue a copy of *count; blocks for the oldest copy when kDepth are in flight.
  // Returns 1 (and sets *value) when a copy has been read, 0 when none has, <0 on error.
  int post(const int32_t* count, hipStream_t st, int32_t* value) {
    int got = 0;
    if (pending_ == kDepth) {
      const int slot = head_ % kDepth;
      IE_HIP(hipEventSynchronize(ev_[slot]));
      *value = words_[slot];
      ++head_;
      --pending_;
      got = 1;
    }
    const int slot = (head_ + pending_) % kDepth;
    IE_HIP(hipMemcpyAsync(&words_[slot], count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    IE_HIP(hipEventRecord(ev_[slot], st));
    ++pending_;
    return got;
  }
  // Read every copy that has already landed, without blocking.
  int drain(int32_t* value) {
    int got = 0;
    while (pending_ > 0) {
      const int slot = head_ % kDepth;
      const hipError_t e = hipEventQuery(ev_[slot]);
      if (e == hipErrorNotReady) break;
      IE_HIP(e);
      *value = words_[slot];
      ++head_;
      --pending_;
      got = 1;
    }
    return got;
  }

 private:
  // One pinned block per host thread, kept for the thread's lifetime (calls on one thread are
  // sequential; calls on different threads do not share it).
  static int32_t* pinned_words() {
    static thread_local int32_t* words = nullptr;
    if (!words && hipHostMalloc((void**)&words, 64 * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      words = nullptr;
    return words;
  }
  int32_t* words_ = nullptr;
  hipEvent_t ev_[kDepth] = {};
  int head_ = 0, pending_ = 0;
};

// Learned warm start: the trunk once per member, then the shift head for every system
// (non-finite starts fall back to zero).  Needs sy.bnorm and sy.sigma.
int stage_warm(Plan& pl, hipStream_t st) {
  Inst& in = pl.in;
  Sys& sy = pl.sy;
  hipLaunchKernelGGL(k_member_features, dim3(nb(in.wmem * in.m)), dim3(256), 0, st, sy.b, sy.ldm, sy.bnorm, in.m,
                     in.wmem, in.wX);
  IE_HIP(hipGetLastError());
  if (in.warm_fp32) IE_TRY(net_forward(*in.net, in.wX, in.wmem, in.m, in.wY, in.wnet, in.wnet_bytes, st));
  else IE_TRY(net_forward_bf16(*in.net, in.wX, in.wmem, in.m, in.wY, in.wnet, in.wnet_bytes, st));
  hipLaunchKernelGGL(k_head_init, dim3((unsigned)sy.S), dim3(256), 0, st, in.wY, in.net->D, in.m, in.wmem, sy.sigma,
                     sy.bnorm, sy.u, sy.ldm, in.fallbacks);
  IE_HIP(hipGetLastError());
  return 0;
}

LMP lmp_of(Plan& pl) {
  LMP l{};
  l.p = pl.pr.p;
  l.Phi = pl.pr.Phi;
  l.SPhi = pl.pr.SPhi;
  l.ld = pl.sy.ldm;
  l.theta = pl.pr.theta;
  l.G = pl.pr.G;
  l.dmin = pl.in.dmin;
  return l;
}

// Multi-shift CG for every member at once (the first sweep of a SOLVER_MULTISHIFT perturbation
// solve): d_s for all systems s = q N + i into sy.x, from the residuals r = b of the base
// systems.  One apply of S per live member per iteration, the same polling as the PCG loop.
int msc_solve(Plan& pl, const Options& op, hipStream_t st) {
  Inst& in = pl.in;
  Sys& sy = pl.sy;
  const int64_t N = in.N;
  const bool od = in.odom();
  double* Vbuf = od ? static_cast<double*>(pl.bf.V) : nullptr;
  const int64_t ldr = ld64(od ? in.m : in.n);
  MscState ms{};
  ms.m = in.m;
  ms.ld = sy.ldm;
  ms.N = N;
  ms.Q = (int)(sy.S / N);
  ms.q0 = op.msc_q0;
  ms.x = sy.x;
  ms.r = sy.r;
  ms.p = sy.p;
  ms.sigma = sy.sigma;
  ms.bnorm = sy.bnorm;
  ms.thresh = sy.thresh;
  ms.zeta = sy.zeta;
  ms.zeta_prev = sy.zeta_prev;
  ms.rr = sy.mrr;
  ms.alpha_prev = sy.malpha;
  ms.beta_prev = sy.mbeta;
  ms.mit = sy.mit;
  ms.relres = sy.rel_in;
  ms.iters = sy.iters;
  ms.done = sy.done;
  ms.flags = in.flags;
  ms.max_iter = op.max_iter;
  const infoesrf_problem* P = in.P;
  int32_t *act_c = sy.act, *nact_c = sy.nact, *act_n = sy.act2, *nact_n = sy.nact2;
  IE_HIP(launch_msc_list(act_c, nact_c, op.msc_q0, N, st));
  IE_HIP(launch_fill_i32(nact_n, 0, 2, st));
  IE_HIP(launch_msc_step(ms, 0, od ? 1 : 0, nullptr, ldr, act_c, nact_c, act_n, nact_n, N, Vbuf, ldr, P->h_ptr,
                         P->h_idx, P->h_w, P->r_var, in.n, st));
  std::swap(act_c, act_n);
  std::swap(nact_c, nact_n);
  LivePoll poll;
  if (op.host_sync) IE_TRY(poll.init());
  int64_t hint = N;
  const int check_every = 4;
  for (int it = 1; it <= op.max_iter; ++it) {
    const int64_t bp = round_up(hint, kSysTile);
    IE_TRY(apply_S(pl, Prec::F64, sy.p, sy.ldm, act_c, nact_c, bp, sy.sigma, nullptr, op.rows_per_wave, st,
                   /*v_ready=*/od, nact_n));
    IE_HIP(launch_msc_step(ms, 1, od ? 1 : 0, static_cast<const double*>(pl.bf.T), ldr, act_c, nact_c, act_n, nact_n,
                           bp, Vbuf, ldr, P->h_ptr, P->h_idx, P->h_w, P->r_var, in.n, st));
    std::swap(act_c, act_n);
    std::swap(nact_c, nact_n);
    if (op.host_sync) {
      int32_t seen = 0;
      int got = poll.drain(&seen);
      IE_TRY(got);
      if (!got && (it % check_every) == 0) {
        got = poll.post(nact_c, st, &seen);
        IE_TRY(got);
      }
      if (got) {
        if (seen == 0) break;
        hint = seen;
      }
    }
  }
  hipLaunchKernelGGL(k_msc_adjust, dim3(1), dim3(256), 0, st, sy.iters, sy.S, sy.mit, N, sy.app_adj);
  IE_HIP(hipGetLastError());
  return 0;
}

// Block PCG for every node at once (the first sweep of a SOLVER_BLOCK perturbation solve): d_s
// for all systems into sy.x from r = b.  Iteration 0 forms P = M R; every later iteration applies
// C to the live nodes' blocks and updates them.
int bcg_solve_all(Plan& pl, const Options& op, hipStream_t st) {
  Inst& in = pl.in;
  Sys& sy = pl.sy;
  const LMP lmp = lmp_of(pl);
  IE_CHECK(sy.bw && sy.bdone, INFOESRF_ERR_HIP, "internal: block solver buffers not allocated");
  BcgState bs{};
  bs.m = in.m;
  bs.ld = sy.ldm;
  bs.N = in.N;
  bs.Q = op.bcg_Q;
  bs.p = lmp.p;
  bs.X = sy.x;
  bs.R = sy.r;
  bs.P = sy.p;
  bs.W = sy.bw;
  bs.Phi = lmp.Phi;
  bs.SPhi = lmp.SPhi;
  bs.ldphi = lmp.ld;
  bs.G = lmp.G;
  bs.theta = lmp.theta;
  bs.dmin = lmp.dmin;
  bs.sigma = sy.sigma;
  bs.thresh = sy.thresh;
  bs.bnorm = sy.bnorm;
  bs.part = sy.bpart;
  bs.nch = bcg_chunks(in.m);
  bs.red = sy.bred;
  bs.coef = sy.bcoef;
  bs.bdone = sy.bdone;
  bs.iters = sy.iters;
  bs.relres = sy.rel_in;
  bs.done = sy.done;
  bs.flags = in.flags;
  bs.max_iter = op.max_iter;
  IE_HIP(launch_fill_i32(sy.bdone, 0, bs.Q, st));
  IE_HIP(launch_bcg_iteration(bs, 0, 0, st));
  LivePoll poll;
  if (op.host_sync) IE_TRY(poll.init());
  int64_t hint = sy.S;
  const int check_every = 2;
  for (int it = 1; it <= op.max_iter + 1; ++it) {
    IE_HIP(launch_bcg_list(sy.bdone, bs.Q, in.N, sy.act, sy.nact, st));
    const int64_t bp = round_up(hint, kSysTile);
    IE_TRY(apply_S(pl, Prec::F64, sy.p, sy.ldm, sy.act, sy.nact, bp, sy.sigma, sy.bw, op.rows_per_wave, st));
    IE_HIP(launch_bcg_iteration(bs, 1, it, st));
    if (op.host_sync) {
      int32_t seen = 0;
      int got = poll.drain(&seen);
      IE_TRY(got);
      if (!got && (it % check_every) == 0) {
        IE_HIP(launch_bcg_list(sy.bdone, bs.Q, in.N, sy.act2, sy.nact2, st));
        got = poll.post(sy.nact2, st, &seen);
        IE_TRY(got);
      }
      if (got) {
        if (seen == 0) break;
        hint = seen;
      }
    }
  }
  return 0;
}

// Iterative refinement around batched PCG.  Solves (1 + sigma_s) u_s + S u_s = b_s for all s.
// Outer sweeps form the true residual r = b - C u in FP64; the inner PCG (apply precision
// op.inner) solves C d = r to the per-system target and u += d.  One inner iteration is two
// launches: the covariance apply on the active columns, and the fused PCG kernel.
// The sweep check's pinned landing place (live count, the call's counters) and its event, one per
// host thread (calls on one thread are sequential), kept for the thread's lifetime.
// The work that consumes u: status (the call's counters and statistics) and output (the
// quadrature sum and the final update).  Both are idempotent.
struct Finalize {
  std::function<int()> status, output;
};

// fin (optional): with host synchronization, each later sweep's check enqueues fin->status and
// copies the counters with the live count, records an event, enqueues fin->output and waits
// only for the event, so the output overlaps the wait and the call can return while it runs;
// *finalized tells whether the last check did this with the final u (then host_stage() holds
// the call's counters), else the caller runs both once more.
// The PCG state of a plan's systems.
PCGState pcg_state_of(Plan& pl, const Options& op) {
  Sys& sy = pl.sy;
  PCGState ps{};
  ps.m = pl.in.m;
  ps.S = sy.S;
  ps.ld = sy.ldm;
  ps.x = sy.x;
  ps.r = sy.r;
  ps.p = sy.p;
  ps.sigma = sy.sigma;
  ps.rz = sy.rz;
  ps.thresh = sy.thresh;
  ps.bnorm = sy.bnorm;
  ps.relres = sy.rel_in;
  ps.iters = sy.iters;
  ps.done = sy.done;
  ps.flags = pl.in.flags;
  ps.max_iter = op.max_iter;
  return ps;
}

// The persistent kernel's in-place apply of S for a plan: the explicit band on the observed
// lattice or the dense S, in FP64 and, for FP32 inner applies, also in FP32 (false for other
// inner precisions, other forms, or a lattice or LDS layout the kernel does not take).  Pointers
// are those of the plan's workspace.
bool tail_inplace(const Plan& pl, const Options& op, TailApply& tap) {
  const Inst& in = pl.in;
  if (op.inner != Prec::F64 && op.inner != Prec::F32) return false;
  if (!in.sd && !(in.obs && in.band)) return false;
  if (in.m > 4096) return false;
  tap = TailApply{};
  tap.kind = in.sd ? 1 : 0;
  tap.g = in.go;
  tap.band = static_cast<const double*>(in.bandO);
  tap.ldb = ld64(in.m);
  tap.S = in.Sd;
  tap.lds = in.lds;
  tap.m = in.m;
  tap.low = op.inner == Prec::F32 ? 1 : 0;
  tap.band32 = in.bandQ32;
  tap.S32 = in.SdQ32;
  return tail_fits(tap);
}

// The zero start of every system of a plan in one launch: the norms of b, u = 0, the per-system
// counters and the first sweep's status (the residual is b itself).
int solve_start(Plan& pl, const Options& op, hipStream_t st) {
  Sys& sy = pl.sy;
  hipLaunchKernelGGL(k_solve_start, dim3((unsigned)sy.Spad), dim3(256), 0, st, sy.b, pl.in.m, sy.ldm, sy.S, sy.bnorm,
                     sy.u, sy.iters, sy.sweeps, sy.fdone, sy.app_adj, op.rtol, op.inner_rtol,
                     op.inner == Prec::F64 ? 1 : 0, op.max_iter, op.fixed > 0 ? 1 : 0, sy.relres, sy.done,
                     sy.thresh, pl.in.flags);
  IE_HIP(hipGetLastError());
  return 0;
}

int stage_solve(Plan& pl, const Options& op, hipStream_t st, const Finalize* fin = nullptr,
                bool* finalized = nullptr) {
  Inst& in = pl.in;
  Sys& sy = pl.sy;
  const int64_t S = sy.S, ldm = sy.ldm, m = in.m;
  const int64_t flat = S * ldm;
  const LMP lmp = lmp_of(pl);
  const bool fp64_inner = (op.inner == Prec::F64);
  const PCGState ps = pcg_state_of(pl, op);

  const bool warm = in.net != nullptr;
  // a zero start forms the norms of b, u = 0, the counters and the first sweep's status in one
  // launch; a learned start first needs the network's u
  const bool fused_start = !warm;
  if (fused_start) {
    IE_TRY(solve_start(pl, op, st));
  } else {
    IE_HIP(launch_col_norms(sy.b, m, S, ldm, sy.bnorm, st));
    IE_HIP(launch_fill_f64(sy.u, 0.0, flat, st));
    IE_TRY(stage_warm(pl, st));
    hipLaunchKernelGGL(k_zero_counters, dim3(nb(sy.Spad)), dim3(256), 0, st, sy.iters, sy.sweeps, sy.fdone, sy.Spad,
                       sy.app_adj);
    IE_HIP(hipGetLastError());
  }
  const bool msc = op.msc_q0 >= 0 && !warm;
  const bool bcg = op.bcg_Q > 0 && !warm;

  // a fixed iteration count is one FP64 inner solve: the status pass after it finishes every system
  const int max_sweeps =
      op.fixed > 0 ? 1 : (op.host_sync ? 40 : (fp64_inner ? 2 : (op.inner == Prec::F32 ? 4 : 10)));
  const int check_every = 4;
  const bool plain = (op.solver == INFOESRF_SOLVER_PLAIN);
  const bool od = in.odom();
  void* Vbuf = od ? pl.bf.V : nullptr;
  // the persistent PCG: FP64 or FP32 inner PCG whose applies it can do in place (each workgroup
  // reads the whole band or S once per iteration, so only those that stay in the L2 of every XCD
  // qualify: at most 1 MiB in the iterations' precision)
  const double elem = op.inner == Prec::F32 ? 4.0 : 8.0;
  const double tail_bytes =
      in.sd ? elem * in.m * in.m : elem * in.m * (2 * in.go.bz + 1) * (2 * in.go.bx + 1);
  TailApply tap{};
  const bool tail_ok = op.tail > 0 && !plain && tail_inplace(pl, op, tap) && tail_bytes <= 1024.0 * 1024;
  // the queue hands out the live systems node by node, smallest shift (the longest solves) first;
  // the perturbation systems share a shift per group of N members, the mean solve is one system
  const int64_t grp = (S % in.N == 0 && S / in.N <= 4096) ? in.N : S;
  // r0 != null: the kernel starts each solve from x = 0 with residual r0 and adds into u;
  // otherwise it continues the batched loop's state
  // the persistent kernel takes every sweep's solve from its start (it needs neither x = 0 nor a
  // copy of the first residual: with a zero start it reads b itself) and then the next sweep's
  // residual and status
  const bool persist = tail_ok && S <= op.tail && !msc && !bcg;
  TailCheck chk{};
  if (persist)
    chk = TailCheck{sy.b, sy.fdone, sy.sweeps, sy.relres, op.rtol, op.fixed > 0 ? 1 : 0, op.inner_rtol, max_sweeps};
  auto run_tail = [&](int32_t* list, int32_t* count, int64_t bound, const double* r0) -> int {
    IE_HIP(launch_order_live(sy.done, sy.sigma, S, grp, list, count, sy.qctr, st));
    IE_HIP(pcg_tail_timed(ps, lmp, tap, list, count, sy.qctr, bound, r0, r0 ? sy.u : nullptr,
                          r0 ? chk : TailCheck{}, st));
    return 0;
  };
  const int64_t ldr = ld64(od ? in.m : in.n);
  int32_t h_nact = (int32_t)S;
  for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
    // outer residual r = b - C u (FP64).  Zero start: the first residual is b itself.  After a
    // persistent solve the kernel has already formed r and the status.
    const bool r_is_b = sweep == 0 && !warm;
    const bool checked = persist && sweep > 0;
    if (r_is_b) {
      if (!persist) {
        hipLaunchKernelGGL(k_copy_f64, dim3(nb(flat)), dim3(256), 0, st, sy.b, sy.r, flat);
        IE_HIP(hipGetLastError());
      }
    } else if (!checked) {
      IE_HIP(launch_compact(sy.fdone, S, sy.act, sy.nact, st));
      IE_TRY(apply_S(pl, Prec::F64, sy.u, ldm, sy.act, sy.nact, S, sy.sigma, sy.q, op.rows_per_wave, st));
      IE_HIP(launch_sub(sy.b, sy.q, sy.r, flat, st));
    }
    const double* rcur = (r_is_b && persist) ? sy.b : sy.r;
    if (!checked && !(sweep == 0 && fused_start)) {
      // the first residual of a zero start is b, whose norms are already there
      const double* rn = r_is_b ? sy.bnorm : sy.rn;
      if (!r_is_b) IE_HIP(launch_col_norms(rcur, m, S, ldm, sy.rn, st));
      hipLaunchKernelGGL(k_sweep_status, dim3(nb(S)), dim3(256), 0, st, rn, sy.bnorm, op.rtol, op.inner_rtol,
                         fp64_inner ? 1 : 0, sy.iters, op.max_iter, op.fixed > 0 ? 1 : 0, sy.relres, sy.fdone,
                         sy.done, sy.thresh, sy.sweeps, (sweep > 0 || warm) ? 1 : 0, S, in.flags);
      IE_HIP(hipGetLastError());
    }
    if (plain) IE_HIP(launch_iota(sy.act, sy.nact, S, st));
    else if (!persist) IE_HIP(launch_compact(sy.done, S, sy.act, sy.nact, st));
    if (finalized) *finalized = false;
    // the persistent kernel needs no live count before the first solve (an empty queue costs
    // microseconds), so that status is not read on the host
    if (op.host_sync && !(persist && sweep == 0)) {
      HostStage* hs = host_stage();
      hipEvent_t ev = host_event();
      IE_CHECK(hs && ev, INFOESRF_ERR_HIP, "pinned host staging or event creation failed");
      const bool spec = fin && sweep > 0;
      // the status kernel of the speculative finish counts the live systems itself
      if (spec) IE_TRY(fin->status());
      else IE_HIP(launch_compact(sy.done, S, sy.act2, sy.nact2, st));
      // one copy of the live count and the counters (the status kernel laid them out as the stage)
      if (spec) IE_HIP(hipMemcpyAsync(hs, sy.stage, sizeof(HostStage), hipMemcpyDeviceToHost, st));
      else IE_HIP(hipMemcpyAsync(&hs->nact, sy.nact2, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      IE_HIP(hipEventRecord(ev, st));
      if (spec) IE_TRY(fin->output());
      IE_HIP(hipEventSynchronize(ev));
      h_nact = hs->nact;
      if (h_nact == 0 || sweep == max_sweeps) {
        if (finalized) *finalized = spec;
        break;
      }
    }
    if (sweep == max_sweeps) break;
    if (persist) {
      // one persistent launch runs every iteration of every live system and adds into u, its
      // sweeps included (the kernel restarts a system from its true residual while that is above
      // rtol and the budget allows); a further launch would skip every system it left
      IE_TRY(run_tail(sy.act, sy.nact, plain ? S : (int64_t)h_nact, rcur));
      break;
    }
    // inner solve on C d = r from d = 0: the multi-shift process first when asked, else PCG
    IE_HIP(launch_fill_f64(sy.x, 0.0, flat, st));
    if ((msc || bcg) && sweep == 0) {
      if (msc) IE_TRY(msc_solve(pl, op, st));
      else IE_TRY(bcg_solve_all(pl, op, st));
      IE_HIP(launch_axpy(sy.u, sy.x, flat, st));
      continue;
    }
    int32_t *act_c = sy.act, *nact_c = sy.nact, *act_n = sy.act2, *nact_n = sy.nact2;
    int64_t hint = plain ? S : (int64_t)h_nact;  // upper bound of the live count on the device
    IE_HIP(launch_fill_i32(nact_n, 0, 2, st));
    IE_HIP(pcg_fused_timed(op.inner, ps, lmp, 0, od ? 1 : 0, plain ? 1 : 0, nullptr, ldr, act_c, nact_c, act_n,
                            nact_n, round_up(hint, kSysTile), Vbuf, ldr, in.P->h_ptr, in.P->h_idx, in.P->h_w,
                            in.P->r_var, in.n, st));
    std::swap(act_c, act_n);
    std::swap(nact_c, nact_n);
    if (tail_ok && hint <= op.tail) {
      // few enough systems left after the first status: one persistent launch runs every
      // iteration from the batched first step
      IE_TRY(run_tail(act_c, nact_c, hint, nullptr));
      IE_HIP(launch_axpy(sy.u, sy.x, flat, st));
      continue;
    }
    LivePoll poll;
    if (op.host_sync) IE_TRY(poll.init());
    for (int it = 1; it <= op.max_iter; ++it) {
      const int64_t bp = round_up(hint, kSysTile);
      // the apply also clears the list counter that the fused kernel fills
      IE_TRY(apply_S(pl, op.inner, sy.p, ldm, act_c, nact_c, bp, sy.sigma, nullptr, op.rows_per_wave, st,
                     /*v_ready=*/od, nact_n));
      IE_HIP(pcg_fused_timed(op.inner, ps, lmp, 1, od ? 1 : 0, plain ? 1 : 0, pl.bf.T, ldr, act_c, nact_c, act_n,
                              nact_n, bp, Vbuf, ldr, in.P->h_ptr, in.P->h_idx, in.P->h_w, in.P->r_var, in.n, st));
      std::swap(act_c, act_n);
      std::swap(nact_c, nact_n);
      if (op.host_sync) {
        // counts only shrink, so any earlier count bounds the current one
        int32_t seen = 0;
        int got = poll.drain(&seen);
        IE_TRY(got);
        if (!got && (it % check_every) == 0) {
          // live count: the compacted list holds exactly the live systems; the masked list
          // keeps every system and counts the live ones separately
          got = poll.post(plain ? nact_c + 1 : nact_c, st, &seen);
          IE_TRY(got);
        }
        if (got) {
          if (seen == 0) break;
          if (!plain) hint = seen;  // compacted lists hold exactly the live systems
          if (tail_ok && seen <= op.tail) {
            // few systems left: one persistent launch iterates each of them to the end
            IE_TRY(run_tail(act_c, nact_c, seen, nullptr));
            break;
          }
        }
      }
    }
    // u += d for every system (d = 0 where the system was not active)
    IE_HIP(launch_axpy(sy.u, sy.x, flat, st));
  }
  return 0;
}

// The device half of finish_status: counters and the caller's per-system statistics.
int finish_enqueue(Plan& pl, const Options& op, infoesrf_stats* stats, int64_t extra_fp64, hipStream_t st) {
  Sys& sy = pl.sy;
  // one block: the counters, the live count for the host check, and the caller's statistics
  int32_t* oi = stats ? stats->iters : nullptr;
  double* orr = stats ? stats->relres : nullptr;
  uint8_t* oc = stats ? stats->converged : nullptr;
  int64_t* out2 = stats ? stats->counters : nullptr;
  hipLaunchKernelGGL(k_finish_counters, dim3(1), dim3(1024), 0, st, sy.iters, sy.sweeps, sy.fdone, sy.S, extra_fp64,
                     sy.app_adj, op.inner == Prec::F64 ? 1 : 0, op.fixed > 0 ? 1 : 0, pl.in.flags, pl.in.fallbacks,
                     pl.in.counters, sy.done, sy.nact2, out2, sy.relres, oi, orr, oc, op.rtol, sy.stage);
  IE_HIP(hipGetLastError());
  return 0;
}

// The host half: with host synchronization, the status code and its message.
int finish_read(Plan& pl, const Options& op, hipStream_t st, const int64_t* staged = nullptr) {
  if (!op.host_sync) return 0;
  int64_t cnt[INFOESRF_NUM_COUNTERS];
  if (staged) {
    std::memcpy(cnt, staged, sizeof(cnt));
  } else {
    IE_HIP(hipMemcpyAsync(cnt, pl.in.counters, sizeof(cnt), hipMemcpyDeviceToHost, st));
    IE_HIP(hipStreamSynchronize(st));
  }
  const int code = (int)cnt[INFOESRF_CNT_STATUS];
  if (code < 0) {
    if (code == INFOESRF_ERR_NOT_SPD) set_error("PCG curvature p^T C p <= 0: localized covariance not PSD");
    else if (code == INFOESRF_ERR_NUMERIC) set_error("non-finite value met during the solve");
    else set_error("invalid input detected on the device");
  } else if (code == INFOESRF_WARN_NOT_CONVERGED) {
    set_error(std::to_string(cnt[INFOESRF_CNT_NOT_CONVERGED]) + " system(s) did not reach rtol");
  }
  return code;
}

int finish_status(Plan& pl, const Options& op, infoesrf_stats* stats, int64_t extra_fp64, hipStream_t st) {
  IE_TRY(finish_enqueue(pl, op, stats, extra_fp64, st));
  return finish_read(pl, op, st);
}

// nnz of H (device) sizes the CSC arrays: the reserved maximum is 64 entries per row on average;
// with host_sync == 1 h_ptr[m] is read and checked against it.

int plan_for(Plan& pl, const infoesrf_problem* P, const Options& op, int64_t S, int64_t nfin, void* ws,
             size_t ws_bytes) {
  Arena ar;
  ar.base = static_cast<char*>(ws);
  plan_layout(pl, ar, P, op, S, nfin);
  const int64_t nnz = nnz_bound(P);
  pl.in.row_of = ar.take<int32_t>(nnz);
  pl.in.w_of = ar.take<double>(nnz);
  pl.bytes = ar.off + 256;
  if (ws) {
    IE_CHECK(ws_bytes >= pl.bytes, INFOESRF_ERR_WORKSPACE,
             "workspace too small: need " + std::to_string(pl.bytes) + " bytes");
  }
  return 0;
}

// ------------------------------------------------------------------ batched instances
// Sum of per-call counter blocks (k blocks of INFOESRF_NUM_COUNTERS); the status is the most
// severe one: any error (the most negative), else the largest warning.
__global__ void k_sum_counters(const int64_t* __restrict__ blocks, int k, int64_t* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= INFOESRF_NUM_COUNTERS) return;
  int64_t acc = 0, worst_err = 0, worst_warn = 0;
  for (int j = 0; j < k; ++j) {
    const int64_t v = blocks[(int64_t)j * INFOESRF_NUM_COUNTERS + c];
    if (c == INFOESRF_CNT_MAX_ITERS) acc = max(acc, v);
    else if (c == INFOESRF_CNT_STATUS) {
      worst_err = min(worst_err, v);
      worst_warn = max(worst_warn, v);
    } else acc += v;
  }
  out[c] = (c == INFOESRF_CNT_STATUS) ? (worst_err < 0 ? worst_err : worst_warn) : acc;
}

// Host worker pool for batched instances: created on first use, kept for the life of the
// process (its threads are detached and end with it).  Each worker owns one non-blocking stream
// per device, so instances on different workers overlap on the GPU.
class WorkerPool {
 public:
  static constexpr int kWorkers = 4;
  static WorkerPool& get() {
    static WorkerPool* pool = new WorkerPool();  // intentionally never destroyed
    return *pool;
  }
  // Runs every task on the workers and returns when all have finished.
  void run(std::vector<std::function<void()>>& tasks) {
    struct Latch {
      std::mutex mu;
      std::condition_variable cv;
      size_t left;
    } latch;
    latch.left = tasks.size();
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& t : tasks)
        q_.push_back([&t, &latch] {
          t();
          std::lock_guard<std::mutex> l2(latch.mu);
          if (--latch.left == 0) latch.cv.notify_all();
        });
    }
    cv_.notify_all();
    std::unique_lock<std::mutex> lk(latch.mu);
    latch.cv.wait(lk, [&] { return latch.left == 0; });
  }
  // Stream idx (< kWorkers) of the calling thread on device dev, created on first use and kept
  // for the thread's lifetime (default priority, non-blocking).
  static hipError_t worker_stream(int dev, int idx, hipStream_t* out) {
    static thread_local std::vector<hipStream_t> streams;
    const size_t k = (size_t)dev * kWorkers + idx;
    if (streams.size() <= k) streams.resize(k + 1, nullptr);
    if (!streams[k]) {
      const hipError_t e = hipStreamCreateWithFlags(&streams[k], hipStreamNonBlocking);
      if (e != hipSuccess) {
        streams[k] = nullptr;
        return e;
      }
    }
    *out = streams[k];
    return hipSuccess;
  }

 private:
  WorkerPool() {
    for (int i = 0; i < kWorkers; ++i) std::thread([this] { loop(); }).detach();
  }
  void loop() {
    for (;;) {
      std::function<void()> job;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return !q_.empty(); });
        job = std::move(q_.front());
        q_.pop_front();
      }
      job();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> q_;
};

// Workspace of one instance: room for its perturbation update and (if asked) its mean update.
size_t instance_ws_bytes(const infoesrf_problem* P, int32_t Q, bool mean, const infoesrf_opts* opts);

// Everything of the perturbation update up to the converged solutions u (Sec. 3.2, eq. E.1):
// validation, set-up, right-hand sides, nodes, preconditioner and the solves.
int perturbation_solve(const infoesrf_problem* prob, int32_t Q, const double* s_nodes, const double* p_weights,
                       const double* y, const infoesrf_opts* opts, Plan& pl, Options& op, void* ws,
                       size_t ws_bytes, hipStream_t st, const Finalize* fin = nullptr,
                       bool* finalized = nullptr) {
  IE_TRY(check_problem(prob));
  IE_TRY(resolve_options(prob, opts, op));
  IE_CHECK(Q >= 1 && Q <= kMaxQ, INFOESRF_ERR_INVALID_ARG, "Q must be in [1, 64]");
  IE_CHECK(s_nodes && p_weights, INFOESRF_ERR_INVALID_ARG, "s_nodes and p_weights must be non-NULL");
  Nodes nd{};
  for (int q = 0; q < Q; ++q) {
    IE_CHECK(std::isfinite(s_nodes[q]) && s_nodes[q] >= 0.0, INFOESRF_ERR_INVALID_ARG, "quadrature nodes must be >= 0");
    IE_CHECK(std::isfinite(p_weights[q]) && p_weights[q] >= 0.0, INFOESRF_ERR_INVALID_ARG,
             "quadrature weights must be >= 0");
    nd.s[q] = s_nodes[q];
    nd.p[q] = p_weights[q];
  }
  IE_CHECK(ws != nullptr, INFOESRF_ERR_WORKSPACE, "workspace is NULL");
  const int64_t N = prob->N;
  const int64_t S = (int64_t)Q * N;
  (void)y;  // the observations do not enter the shifted systems' solutions
  if (op.solver == INFOESRF_SOLVER_MULTISHIFT) {
    // the base is the smallest node (the worst conditioned system, which converges last); the
    // process has no preconditioner, and later correction sweeps use plain PCG
    int q0 = 0;
    for (int q = 1; q < Q; ++q)
      if (nd.s[q] < nd.s[q0]) q0 = q;
    op.msc_q0 = q0;
    op.p = 0;
    op.k = 0;
  }
  if (op.solver == INFOESRF_SOLVER_BLOCK) op.bcg_Q = Q;
  IE_TRY(plan_for(pl, prob, op, S, N, ws, ws_bytes));
  IE_TRY(stage_setup(pl, op, st));
  Sys& sy = pl.sy;
  IE_HIP(launch_obs_rhs_padded(prob->h_ptr, prob->h_idx, prob->h_w, prob->r_var, pl.in.Z, pl.in.n, N, pl.in.m, sy.b,
                               sy.ldm, S, sy.Spad, st));
  hipLaunchKernelGGL(k_set_nodes, dim3(nb(std::max<int64_t>(sy.Spad, kMaxQ))), dim3(256), 0, st, nd, Q, N, sy.sigma,
                     sy.pw, (int64_t)0, 0.0, sy.Spad);
  IE_HIP(hipGetLastError());
  IE_TRY(stage_precond(pl, op, st));
  IE_TRY(stage_solve(pl, op, st, fin, finalized));
  return 0;
}

// ------------------------------------------------------------------ batched instances, one launch
// Every instance's systems (Q N perturbation systems and, when its mean is wanted, the mean system
// at shift 0, all in one plan) in one persistent launch per sweep (Sec. 3.2: the (q, i) systems are
// independent).  Set-up per instance on the caller's stream, then per sweep the queue over every
// instance's live systems and the launch, then per instance the quadrature sum, the final update
// and the counters.  Taken when every instance's inner solve can run in the persistent kernel.

// Workspace of one instance on this path (its mean system included).
size_t combined_ws_bytes(const infoesrf_problem* P, int32_t Q, const infoesrf_opts* o) {
  Options op;
  if (check_problem(P) < 0 || resolve_options(P, o, op) < 0) return 0;
  if (Q < 1 || Q > kMaxQ) return 0;
  Plan pl;
  if (plan_for(pl, P, op, (int64_t)Q * P->N + 1, P->N + 1, nullptr, 0) < 0) return 0;
  return pl.bytes;
}

// Whether every instance qualifies: the compacted PCG solver from a zero start, the persistent
// kernel allowed (tail_systems >= 0), FP64 or FP32 inner applies done in place, m <= 4096, and one
// preconditioner size for all.
bool batch_one_launch(const infoesrf_problem* probs, int count, const int32_t* Q,
                      const std::vector<infoesrf_opts>& oj) {
  int p = -1;
  for (int j = 0; j < count; ++j) {
    const infoesrf_opts& o = oj[j];
    if (o.solver != INFOESRF_SOLVER_COMPACT || o.warm_start != INFOESRF_START_ZERO || o.tail_systems < 0)
      return false;
    Options op;
    if (check_problem(&probs[j]) < 0 || resolve_options(&probs[j], &o, op) < 0) return false;
    if (Q[j] < 1 || Q[j] > kMaxQ || (int64_t)Q[j] * probs[j].N + 1 >= (int64_t(1) << kTailSysBits)) return false;
    Plan pl;
    if (plan_for(pl, &probs[j], op, (int64_t)Q[j] * probs[j].N + 1, probs[j].N + 1, nullptr, 0) < 0) return false;
    TailApply tap;
    if (!tail_inplace(pl, op, tap)) return false;
    if (p >= 0 && op.p != p) return false;
    p = op.p;
  }
  clear_error();
  return true;
}

// Batch-level arrays after the instances' slices: descriptors, queue scratch and the summed
// counters.
struct BatchArea {
  TailInst* table;
  int32_t *seg, *list, *cnt, *words;  // words: live count and queue counter of each class
  int64_t* total;                     // summed counters
  size_t bytes;
};
BatchArea batch_area(char* base, int count, int64_t systems) {
  Arena ar;
  ar.base = base;
  BatchArea b{};
  b.table = ar.take<TailInst>(count);
  b.seg = ar.take<int32_t>(systems);
  b.list = ar.take<int32_t>(systems);
  b.cnt = ar.take<int32_t>(count);
  b.words = ar.take<int32_t>(6);  // three classes
  b.total = ar.take<int64_t>(INFOESRF_NUM_COUNTERS);
  b.bytes = ar.off + 256;
  return b;
}

// The message of a status code from the device counters.
std::string status_message(int code, int64_t not_converged) {
  if (code == INFOESRF_ERR_NOT_SPD) return "PCG curvature p^T C p <= 0: localized covariance not PSD";
  if (code == INFOESRF_ERR_NUMERIC) return "non-finite value met during the solve";
  if (code < 0) return "invalid input detected on the device (observation operator, r_var or X)";
  if (code == INFOESRF_WARN_NOT_CONVERGED) return std::to_string(not_converged) + " system(s) did not reach rtol";
  return "";
}

int batched_one_launch(const infoesrf_problem* probs, int count, const int32_t* Q, const double* const* s_nodes,
                       const double* const* p_weights, const double* const* y, double* const* mean_a,
                       double* const* Xa_pert, std::vector<infoesrf_opts>& oj, infoesrf_stats* stats, char* base,
                       const std::vector<size_t>& off, const std::vector<int64_t>& sys_off, int64_t* cnt,
                       const BatchArea& ba, const std::vector<int>& order, bool host_sync, hipStream_t st) {
  std::vector<Plan> pl(count);
  std::vector<Options> op(count);
  std::vector<TailInst> desc(count);
  std::vector<char> mean(count, 0);
  std::vector<int> codes(count, 0);
  std::vector<std::string> msgs(count);
  // one instance's set-up on stream ss, without host reads (inputs that fail the device's checks
  // set its flags, reported through its counters); an instance that fails on the host is left
  // out of the launches and reported
  auto setup = [&](int j, hipStream_t ss) -> int {
    const infoesrf_problem* P = &probs[j];
    const int64_t N = P->N, QN = (int64_t)Q[j] * N;
    mean[j] = (mean_a && mean_a[j]) ? 1 : 0;
    const int64_t S = QN + mean[j];
    IE_TRY(resolve_options(P, &oj[j], op[j]));
    op[j].host_sync = 0;
    IE_TRY(plan_for(pl[j], P, op[j], S, N + mean[j], base + off[j], off[j + 1] - off[j]));
    Nodes nd{};
    for (int q = 0; q < Q[j]; ++q) {
      IE_CHECK(std::isfinite(s_nodes[j][q]) && s_nodes[j][q] >= 0.0 && std::isfinite(p_weights[j][q]) &&
                   p_weights[j][q] >= 0.0,
               INFOESRF_ERR_INVALID_ARG, "quadrature nodes and weights must be >= 0");
      nd.s[q] = s_nodes[j][q];
      nd.p[q] = p_weights[j][q];
    }
    Plan& p = pl[j];
    Sys& sy = p.sy;
    IE_TRY(stage_setup(p, op[j], ss));
    IE_HIP(launch_obs_rhs_padded(P->h_ptr, P->h_idx, P->h_w, P->r_var, p.in.Z, p.in.n, N, p.in.m, sy.b, sy.ldm, QN,
                                 sy.Spad, ss));
    if (mean[j])
      IE_HIP(launch_innovation(P->h_ptr, P->h_idx, P->h_w, P->r_var, y[j], p.in.mu, p.in.m, p.in.n, sy.b, sy.ldm, QN,
                               ss));
    hipLaunchKernelGGL(k_set_nodes, dim3(nb(std::max<int64_t>(sy.Spad, kMaxQ))), dim3(256), 0, ss, nd, Q[j], N,
                       sy.sigma, sy.pw, (int64_t)mean[j], 0.0, sy.Spad);
    IE_HIP(hipGetLastError());
    IE_TRY(stage_precond(p, op[j], ss));
    IE_TRY(solve_start(p, op[j], ss));
    TailInst& d = desc[j];
    d.st = pcg_state_of(p, op[j]);
    d.lmp = lmp_of(p);
    IE_CHECK(tail_inplace(p, op[j], d.ap), INFOESRF_ERR_INVALID_ARG, "no in-place apply for the persistent kernel");
    const int budget = op[j].fixed > 0 ? 1 : (host_sync ? 40 : (op[j].inner == Prec::F64 ? 2 : 4));
    d.chk = TailCheck{sy.b, sy.fdone, sy.sweeps, sy.relres, op[j].rtol, op[j].fixed > 0 ? 1 : 0,
                      op[j].inner_rtol, budget};
    d.r0 = sy.b;  // the first sweep's residual (zero start)
    d.uacc = sy.u;
    d.grp = (int32_t)N;
    return 0;
  };
  // the set-ups fork from `st` over the worker streams and join back (capture safe)
  int dev = 0;
  IE_HIP(hipGetDevice(&dev));
  struct Events {
    std::vector<hipEvent_t> e;
    ~Events() {
      for (auto x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev;
  const int nw = std::min<int>(WorkerPool::kWorkers, count);
  ev.e.assign(1 + nw, nullptr);
  for (auto& x : ev.e) IE_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
  IE_HIP(hipEventRecord(ev.e[0], st));
  std::vector<hipStream_t> ws(nw);
  for (int w = 0; w < nw; ++w) {
    IE_HIP(WorkerPool::worker_stream(dev, w, &ws[w]));
    IE_HIP(hipStreamWaitEvent(ws[w], ev.e[0], 0));
  }
  std::vector<int> live;  // instances in the launches, largest first
  for (int k = 0; k < count; ++k) {
    const int j = order[k];
    codes[j] = setup(j, ws[k % nw]);
    if (codes[j] < 0) msgs[j] = g_last_error;
    else live.push_back(j);
  }
  for (int w = 0; w < nw; ++w) {
    IE_HIP(hipEventRecord(ev.e[1 + w], ws[w]));
    IE_HIP(hipStreamWaitEvent(st, ev.e[1 + w], 0));
  }
  // one launch per shape of the kernel (rows a thread and workgroup size, from m): the larger
  // instances first, each class with its slice of the table, the queue's scratch and its counters
  // (m <= 512 on 256-thread workgroups, several a CU, rather than leaving most of a 1024-row
  // workgroup idle)
  std::vector<int> big, mid, small;
  for (int j : live) (probs[j].m > 1024 ? big : (probs[j].m > 512 ? mid : small)).push_back(j);
  std::vector<std::vector<int>> classes;
  for (const auto* cl : {&big, &mid, &small})
    if (!cl->empty()) classes.push_back(*cl);
  const int nl = (int)live.size();
  // one launch per class runs every sweep: each workgroup iterates a system to its inner target,
  // adds the correction into u, checks the true FP64 residual and, while that is above rtol and
  // the instance's sweep budget allows, restarts from it at once.  A system that spends its
  // budget stays live and is reported not converged; a further launch would skip it.
  if (nl > 0) {
    int t0 = 0;
    int64_t s0 = 0;
    for (size_t c = 0; c < classes.size(); ++c) {
      const std::vector<int>& cl = classes[c];
      std::vector<TailInst> ordered(cl.size());
      int64_t segc = 0;
      for (size_t k = 0; k < cl.size(); ++k) {
        ordered[k] = desc[cl[k]];
        ordered[k].seg = segc;
        segc += ordered[k].st.S;
      }
      // the launch writes the table, builds the queue (live systems instance by instance,
      // largest first) and iterates
      IE_HIP(launch_pcg_tail_multi(ordered.data(), (int)cl.size(), ba.table + t0, ba.seg + s0, ba.cnt + t0,
                                   ba.list + s0, ba.words + 2 * c, ba.words + 2 * c + 1, segc, st));
      t0 += (int)cl.size();
      s0 += segc;
    }
  }
  // per instance: u_bar_i = sum_q p_q u_{q,i} (and the mean's u as column N), the final updates
  // and the counters
  for (int k = 0; k < nl; ++k) {
    const int j = live[k];
    Plan& p = pl[j];
    Sys& sy = p.sy;
    const int64_t N = probs[j].N, QN = (int64_t)Q[j] * N;
    IE_HIP(launch_quad_combine(sy.u, sy.ldm, p.in.m, N, Q[j], sy.pw, p.fn.ubar, sy.ldm, 0, p.fn.act, p.fn.nact, st));
    if (mean[j]) {
      IE_HIP(launch_copy_cols(sy.u + QN * sy.ldm, sy.ldm, p.in.m, 1, p.fn.ubar + N * sy.ldm, sy.ldm, st));
      IE_HIP(launch_iota(p.fn.act, p.fn.nact, N + 1, st));
    }
    IE_TRY(apply_state(p, p.fn.ubar, sy.ldm, p.fn.act, p.fn.nact, N + mean[j], op[j].rows_per_wave, st));
    IE_HIP(launch_final_pert(p.in.Z, (const double*)p.bf.T, ld64(p.in.n), p.in.n, N, std::sqrt((double)(N - 1)),
                             Xa_pert[j], st));
    if (mean[j]) IE_HIP(launch_final_mean(p.in.mu, (const double*)p.bf.T, ld64(p.in.n), p.in.n, N, mean_a[j], st));
    infoesrf_stats sj{};
    if (stats) {
      sj.iters = stats->iters ? stats->iters + sys_off[j] : nullptr;
      sj.relres = stats->relres ? stats->relres + sys_off[j] : nullptr;
      sj.converged = stats->converged ? stats->converged + sys_off[j] : nullptr;
    }
    sj.counters = cnt + (int64_t)(2 * j) * INFOESRF_NUM_COUNTERS;
    IE_TRY(finish_enqueue(p, op[j], &sj, 2 * p.pr.k + N + mean[j], st));
  }
  hipLaunchKernelGGL(k_sum_counters, dim3(1), dim3(64), 0, st, cnt, 2 * count, ba.total);
  IE_HIP(hipGetLastError());
  if (stats && stats->counters)
    IE_HIP(hipMemcpyAsync(stats->counters, ba.total, sizeof(int64_t) * INFOESRF_NUM_COUNTERS,
                          hipMemcpyDeviceToDevice, st));
  if (!host_sync) {
    for (int j = 0; j < count; ++j)
      if (codes[j] < 0) {
        set_error("instance " + std::to_string(j) + ": " + msgs[j]);
        return codes[j];
      }
    return 0;
  }
  // the instances' own counters name the first that failed on the device
  std::vector<int64_t> blocks((size_t)2 * count * INFOESRF_NUM_COUNTERS);
  int64_t tot[INFOESRF_NUM_COUNTERS];
  IE_HIP(hipMemcpyAsync(blocks.data(), cnt, sizeof(int64_t) * blocks.size(), hipMemcpyDeviceToHost, st));
  IE_HIP(hipMemcpyAsync(tot, ba.total, sizeof(tot), hipMemcpyDeviceToHost, st));
  IE_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < count; ++j) {
    const int64_t* bj = blocks.data() + (size_t)2 * j * INFOESRF_NUM_COUNTERS;
    const int cj = codes[j] < 0 ? codes[j] : (int)bj[INFOESRF_CNT_STATUS];
    if (cj < 0) {
      set_error("instance " + std::to_string(j) + ": " +
                (codes[j] < 0 ? msgs[j] : status_message(cj, bj[INFOESRF_CNT_NOT_CONVERGED])));
      return cj;
    }
  }
  const int code = (int)tot[INFOESRF_CNT_STATUS];
  if (code != 0) set_error(status_message(code, tot[INFOESRF_CNT_NOT_CONVERGED]));
  return code;
}

}  // namespace
}  // namespace infoesrf

using namespace infoesrf;

namespace infoesrf {

int cov_apply_run(const infoesrf_problem* prob, const double* V, int64_t ldv, int64_t B, double* PV, int64_t ldpv,
                  const Options& op, void* ws, hipStream_t st);

// ------------------------------------------------------------------ no-allocation scratch
// The workspace of infoesrf_cov_apply_noalloc: one array per device, held from the library's
// load until the process ends.  In host code `scratch` names a host-side stand-in, never a device
// address: kernels and copies get the address hipGetSymbolAddress returns for the current device,
// looked up on the first call on that device and kept.  Calls that overlap on one device share
// the array and race.
static __device__ __align__(256) unsigned char scratch[INFOESRF_NOALLOC_SCRATCH_BYTES];
constexpr int kNoAllocDevices = 64;
std::atomic<void*> g_scratch_addr[kNoAllocDevices];

int noalloc_scratch(void** out) {
  int dev = -1;
  IE_HIP(hipGetDevice(&dev));
  IE_CHECK(dev >= 0 && dev < kNoAllocDevices, INFOESRF_ERR_INVALID_ARG,
           "infoesrf_cov_apply_noalloc: device index beyond " + std::to_string(kNoAllocDevices));
  void* p = g_scratch_addr[dev].load();
  if (!p) {
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    IE_CHECK(e == hipSuccess && p != nullptr, INFOESRF_ERR_HIP,
             std::string("hipGetSymbolAddress of the no-allocation scratch failed: ") + hipGetErrorString(e));
    g_scratch_addr[dev].store(p);  // the same address if two first calls race
  }
  *out = p;
  return 0;
}

}  // namespace infoesrf

extern "C" {

void infoesrf_default_opts(infoesrf_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-8;
  o->inner_rtol = 0.0;
  o->max_iter = 1000;
  o->n_ritz = 10;
  o->oversample = 10;
  o->precision = INFOESRF_FP64;
  o->solver = INFOESRF_SOLVER_COMPACT;
  o->warm_start = INFOESRF_START_ZERO;
  o->host_sync = 1;
  o->apply_domain = INFOESRF_DOMAIN_STATE;
  o->seed = 0x2503002530ULL;
}

const char* infoesrf_error_string(int code) {
  switch (code) {
    case INFOESRF_OK: return "ok";
    case INFOESRF_WARN_NOT_CONVERGED: return "some systems did not reach the residual tolerance";
    case INFOESRF_ERR_INVALID_ARG: return "invalid argument";
    case INFOESRF_ERR_NOT_SPD: return "matrix not symmetric positive definite (PCG breakdown)";
    case INFOESRF_ERR_NUMERIC: return "non-finite value (NaN or Inf)";
    case INFOESRF_ERR_WORKSPACE: return "workspace missing or too small";
    case INFOESRF_ERR_HIP: return "HIP runtime error";
    default: return "unknown status code";
  }
}

const char* infoesrf_last_error(void) { return g_last_error.c_str(); }

size_t infoesrf_workspace_bytes(const infoesrf_problem* prob, int32_t Q, const infoesrf_opts* opts) {
  clear_error();
  if (check_problem(prob) < 0) return 0;
  Options op;
  if (resolve_options(prob, opts, op) < 0) return 0;
  if (Q < 0 || Q > kMaxQ) {
    set_error("Q must be in [0, 64]");
    return 0;
  }
  Plan pl;
  const int64_t S = Q > 0 ? (int64_t)Q * prob->N : 1;
  const int64_t nfin = Q > 0 ? prob->N : 1;
  if (plan_for(pl, prob, op, S, nfin, nullptr, 0) < 0) return 0;
  return pl.bytes;
}

size_t infoesrf_cov_apply_workspace_bytes(const infoesrf_problem* prob, int64_t B, const infoesrf_opts* opts) {
  clear_error();
  if (check_problem(prob) < 0) return 0;
  Options op;
  if (resolve_options(prob, opts, op) < 0) return 0;
  const int64_t cols = std::max<int64_t>(B, 1);
  const int64_t ldr = ld64(prob->n);
  Arena ar;
  ar.take<double>(prob->n);                  // mu
  ar.take<double>(prob->n * prob->N);        // Z
  ar.take<float>(prob->n * prob->N);         // Z32
  ar.take<float>((2 * prob->loc.bz + 1) * (2 * prob->loc.bx + 1));
  ar.take<float>(ldr * cols);                // low-precision V
  ar.take<float>(ldr * cols);                // FP32 T
  if (op.band) ar.take<double>((int64_t)(2 * prob->loc.bz + 1) * (2 * prob->loc.bx + 1) * ldr);  // band
  return ar.off + 256;
}

int infoesrf_cov_apply(const infoesrf_problem* prob, const double* V, int64_t ldv, int64_t B, double* PV,
                       int64_t ldpv, const infoesrf_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  IE_TRY(check_problem(prob));
  Options op;
  IE_TRY(resolve_options(prob, opts, op));
  IE_CHECK(B >= 0, INFOESRF_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0) return INFOESRF_OK;
  IE_CHECK(V && PV, INFOESRF_ERR_INVALID_ARG, "V and PV must be non-NULL");
  IE_CHECK(ldv >= prob->n && ldpv >= prob->n, INFOESRF_ERR_INVALID_ARG, "ldv and ldpv must be >= n");
  IE_CHECK(ws != nullptr, INFOESRF_ERR_WORKSPACE, "workspace is NULL");
  const size_t need = infoesrf_cov_apply_workspace_bytes(prob, B, opts);
  IE_CHECK(ws_bytes >= need, INFOESRF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  return infoesrf::cov_apply_run(prob, V, ldv, B, PV, ldpv, op, ws, static_cast<hipStream_t>(stream));
}

int infoesrf_cov_apply_noalloc(const infoesrf_problem* prob, const double* V, int64_t ldv, int64_t B, double* PV,
                               int64_t ldpv, const infoesrf_opts* opts, void* stream) {
  clear_error();
  IE_TRY(check_problem(prob));
  Options op;
  IE_TRY(resolve_options(prob, opts, op));
  IE_CHECK(B >= 0, INFOESRF_ERR_INVALID_ARG, "B must be >= 0");
  if (B == 0) return INFOESRF_OK;
  IE_CHECK(V && PV, INFOESRF_ERR_INVALID_ARG, "V and PV must be non-NULL");
  IE_CHECK(ldv >= prob->n && ldpv >= prob->n, INFOESRF_ERR_INVALID_ARG, "ldv and ldpv must be >= n");
  const size_t need = infoesrf_cov_apply_workspace_bytes(prob, B, opts);
  IE_CHECK(need > 0 && need <= INFOESRF_NOALLOC_SCRATCH_BYTES, INFOESRF_ERR_WORKSPACE,
           "infoesrf_cov_apply_noalloc: this call needs " + std::to_string(need) +
               " bytes of scratch, above its fixed " + std::to_string((size_t)INFOESRF_NOALLOC_SCRATCH_BYTES) +
               " (use infoesrf_cov_apply with a caller workspace, or fewer columns per call)");
  void* ws = nullptr;
  IE_TRY(infoesrf::noalloc_scratch(&ws));
  return infoesrf::cov_apply_run(prob, V, ldv, B, PV, ldpv, op, ws, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace infoesrf {

// The body of infoesrf_cov_apply on a workspace of at least infoesrf_cov_apply_workspace_bytes:
// every word of it that the call reads is written by the call first, so its contents on entry do
// not matter.
int cov_apply_run(const infoesrf_problem* prob, const double* V, int64_t ldv, int64_t B, double* PV, int64_t ldpv,
                  const Options& op, void* ws, hipStream_t st) {
  const int64_t n = prob->n, N = prob->N;
  const int64_t ldr = ld64(n);
  Arena ar;
  ar.base = static_cast<char*>(ws);
  double* mu = ar.take<double>(n);
  double* Z = ar.take<double>(n * N);
  float* Z32 = ar.take<float>(n * N);
  float* tab32 = ar.take<float>((2 * prob->loc.bz + 1) * (2 * prob->loc.bx + 1));
  void* Vlow = ar.take<float>(ldr * B);
  float* T32 = ar.take<float>(ldr * B);
  void* band = op.band ? ar.take<double>((int64_t)(2 * prob->loc.bz + 1) * (2 * prob->loc.bx + 1) * ldr) : nullptr;
  const bool low = op.inner != Prec::F64;
  IE_HIP(launch_ens_stats(prob->X, n, N, mu, Z, low ? Z32 : nullptr, st));
  if (op.band) {
    const infoesrf_loc& L = prob->loc;
    const Grid g{L.nz, L.nx, L.periodic_z, L.periodic_x, L.bz, L.bx, L.table, nullptr, nullptr};
    // the FP32 band fits in the FP64 band's storage
    IE_HIP(launch_band_build(op.inner, g, Z, n, N, band, ldr, st));
    if (!low) {
      IE_HIP(cov_band_timed(Prec::F64, g, band, ldr, V, ldv, B, B, nullptr, PV, ldpv, st));
    } else {
      float* V32 = static_cast<float*>(Vlow);
      hipLaunchKernelGGL((k_convert_cols<double, float>), dim3(nb(ldr * B)), dim3(256), 0, st, V, ldv, n, B, V32,
                         ldr, 1);
      IE_HIP(hipGetLastError());
      IE_HIP(cov_band_timed(Prec::F32, g, band, ldr, V32, ldr, B, B, nullptr, T32, ldr, st));
      hipLaunchKernelGGL((k_convert_cols<float, double>), dim3(nb(ldpv * B)), dim3(256), 0, st, T32, ldr, n, B, PV,
                         ldpv, 0);
      IE_HIP(hipGetLastError());
    }
  } else if (prob->loc.kind == INFOESRF_LOC_DENSE) {
    IE_CHECK(!low, INFOESRF_ERR_INVALID_ARG, "dense localization supports FP64 only");
    IE_HIP(launch_cov_dense(prob->loc.dense, Z, n, N, V, ldv, B, PV, ldpv, st));
  } else {
    const infoesrf_loc& L = prob->loc;
    Grid g{L.nz, L.nx, L.periodic_z, L.periodic_x, L.bz, L.bx, L.table, tab32, nullptr};
    if (!low) {
      // column-major V and PV are system-major apply buffers already
      IE_HIP(cov_stencil_timed(Prec::F64, g, Z, n, N, V, ldv, B, B, nullptr, PV, ldpv,
                               tile_for(op.rows_per_wave, B, op_key(1, Prec::F64, g, N)), st));
    } else {
      IE_HIP(launch_convert_f32(L.table, tab32, (int64_t)(2 * L.bz + 1) * (2 * L.bx + 1), st));
      if (op.inner == Prec::BF16) {
        __hip_bfloat16* V16 = static_cast<__hip_bfloat16*>(Vlow);
        hipLaunchKernelGGL((k_convert_cols<double, __hip_bfloat16>), dim3(nb(ldr * B)), dim3(256), 0, st, V, ldv, n,
                           B, V16, ldr, 1);
        IE_HIP(hipGetLastError());
        IE_HIP(cov_bf16_timed(g, Z32, n, N, V16, ldr, B, B, nullptr, T32, ldr, tile_for_bf16(op.rows_per_wave, B, op_key(2, Prec::BF16, g, N)),
                              st));
      } else {
        float* V32 = static_cast<float*>(Vlow);
        hipLaunchKernelGGL((k_convert_cols<double, float>), dim3(nb(ldr * B)), dim3(256), 0, st, V, ldv, n, B, V32,
                           ldr, 1);
        IE_HIP(hipGetLastError());
        IE_HIP(cov_stencil_timed(Prec::F32, g, Z32, n, N, V32, ldr, B, B, nullptr, T32, ldr,
                                 tile_for(op.rows_per_wave, B, op_key(1, Prec::F64, g, N)), st));
      }
      hipLaunchKernelGGL((k_convert_cols<float, double>), dim3(nb(ldpv * B)), dim3(256), 0, st, T32, ldr, n, B, PV,
                         ldpv, 0);
      IE_HIP(hipGetLastError());
    }
  }
  if (op.host_sync) IE_HIP(hipStreamSynchronize(st));
  return INFOESRF_OK;
}

}  // namespace infoesrf

extern "C" {

int infoesrf_mean_update(const infoesrf_problem* prob, const double* y, double* mean_a, const infoesrf_opts* opts,
                         infoesrf_stats* stats, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  IE_TRY(check_problem(prob));
  Options op;
  IE_TRY(resolve_options(prob, opts, op));
  IE_CHECK(y && mean_a, INFOESRF_ERR_INVALID_ARG, "y and mean_a must be non-NULL");
  IE_CHECK(ws != nullptr, INFOESRF_ERR_WORKSPACE, "workspace is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Plan pl;
  IE_TRY(plan_for(pl, prob, op, 1, 1, ws, ws_bytes));
  IE_TRY(stage_setup(pl, op, st));
  Sys& sy = pl.sy;
  IE_HIP(launch_fill_f64(sy.b, 0.0, sy.ldm * sy.Spad, st));
  IE_HIP(launch_innovation(prob->h_ptr, prob->h_idx, prob->h_w, prob->r_var, y, pl.in.mu, pl.in.m, pl.in.n, sy.b,
                           sy.ldm, 0, st));
  IE_HIP(launch_fill_f64(sy.sigma, 0.0, sy.Spad, st));
  IE_TRY(stage_precond(pl, op, st));
  IE_TRY(stage_solve(pl, op, st));
  // mean_a = mu + P H^T R^{-1/2} u0
  IE_HIP(launch_iota(pl.fn.act, pl.fn.nact, 1, st));
  IE_TRY(apply_state(pl, sy.u, sy.ldm, pl.fn.act, pl.fn.nact, 1, op.rows_per_wave, st));
  IE_HIP(launch_final_mean(pl.in.mu, (const double*)pl.bf.T, ld64(pl.in.n), pl.in.n, 0, mean_a, st));
  return finish_status(pl, op, stats, 2 * pl.pr.k + 1, st);
}

int infoesrf_perturbation_update(const infoesrf_problem* prob, int32_t Q, const double* s_nodes,
                                 const double* p_weights, const double* y, double* Xa_pert,
                                 const infoesrf_opts* opts, infoesrf_stats* stats, void* ws, size_t ws_bytes,
                                 void* stream) {
  clear_error();
  IE_CHECK(Xa_pert, INFOESRF_ERR_INVALID_ARG, "Xa_pert must be non-NULL");
  Plan pl;
  Options op;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t N = prob->N;
  // u_bar_i = sum_q p_q u_{q,i}; Xa_pert = sqrt(N-1) (Z - P H^T R^{-1/2} U_bar); idempotent, so
  // the solve may enqueue it before its last status read and again if a later sweep changes u
  Finalize fin;
  fin.status = [&]() -> int { return finish_enqueue(pl, op, stats, 2 * pl.pr.k + N, st); };
  fin.output = [&]() -> int {
    Sys& sy = pl.sy;
    IE_HIP(
        launch_quad_combine(sy.u, sy.ldm, pl.in.m, N, Q, sy.pw, pl.fn.ubar, sy.ldm, 0, pl.fn.act, pl.fn.nact, st));
    IE_TRY(apply_state(pl, pl.fn.ubar, sy.ldm, pl.fn.act, pl.fn.nact, N, op.rows_per_wave, st));
    IE_HIP(launch_final_pert(pl.in.Z, (const double*)pl.bf.T, ld64(pl.in.n), pl.in.n, N,
                             std::sqrt((double)(N - 1)), Xa_pert, st));
    return 0;
  };
  bool finalized = false;
  IE_TRY(perturbation_solve(prob, Q, s_nodes, p_weights, y, opts, pl, op, ws, ws_bytes, st, &fin, &finalized));
  if (finalized) return finish_read(pl, op, st, host_stage()->cnt);  // counters came with the last check
  IE_TRY(fin.status());
  IE_TRY(fin.output());
  return finish_read(pl, op, st);
}

int infoesrf_autotune(const infoesrf_problem* prob, int32_t Q, const infoesrf_opts* opts, void* ws,
                      size_t ws_bytes, void* stream, int32_t* report) {
  clear_error();
  IE_TRY(check_problem(prob));
  Options op;
  IE_TRY(resolve_options(prob, opts, op));
  IE_CHECK(Q >= 0 && Q <= kMaxQ, INFOESRF_ERR_INVALID_ARG, "Q must be in [0, 64]");
  IE_CHECK(ws != nullptr, INFOESRF_ERR_WORKSPACE, "workspace is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t S = Q > 0 ? (int64_t)Q * prob->N : 1;
  Plan pl;
  IE_TRY(plan_for(pl, prob, op, S, Q > 0 ? prob->N : 1, ws, ws_bytes));
  op.host_sync = 1;  // the tuner reads timings on the host
  IE_TRY(stage_setup(pl, op, st, /*solve=*/false));
  Inst& in = pl.in;
  IE_CHECK(!in.dense, INFOESRF_ERR_INVALID_ARG, "dense localization has nothing to tune");
  const Grid& g = in.obs ? in.go : in.gs;
  const int64_t rows = in.obs ? in.m : in.n;
  const int64_t ldr = ld64(rows);
  const int64_t cols = pl.bf.cols;
  IE_HIP(launch_fill_f64((double*)pl.bf.V, 1.0, ldr * cols, st));
  // the inner precision's apply, and the FP64 apply of the residual sweeps when they differ
  // (with a dense S, applies of P are FP64 only: they form S and the final state-space update)
  std::vector<Prec> precs{in.sd ? Prec::F64 : op.inner};
  if (precs[0] != Prec::F64) precs.push_back(Prec::F64);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  IE_HIP(hipEventCreate(&e0));
  IE_HIP(hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  int rep = 0;
  for (Prec prec : precs) {
    const bool band = in.band;
    const int form = band ? 0 : (prec == Prec::BF16 ? 2 : 1);
    const TuneKey key = band ? TuneKey{0, prec == Prec::F64 ? 0 : 1, g.nz, g.nx, g.bz, g.bx, 0}
                             : op_key(form, prec, g, in.N);
    const size_t es = prec == Prec::F64 ? 8 : 4;
    std::vector<int> cands;
    if (band) {
      for (int c : {8, 16, 32, 64})
        if ((size_t)c * (64 + 2 * g.bx) * es <= 150 * 1024) cands.push_back(c);
    } else {
      cands = {16, 32, 64, 128};
    }
    const void* bandp = in.obs ? (prec == Prec::F64 ? in.bandO : in.bandO32) : (prec == Prec::F64 ? in.bandS : in.bandS32);
    const void* Zu = (prec == Prec::F64) ? (in.obs ? (const void*)in.Zt : (const void*)in.Z)
                                         : (in.obs ? (const void*)in.Zt32 : (const void*)in.Z32);
    auto launch = [&](int64_t B) -> hipError_t {
      if (band) return launch_band_apply(prec, g, bandp, ldr, pl.bf.V, ldr, cols, B, nullptr, pl.bf.T, ldr, st);
      if (prec == Prec::BF16)
        return launch_cov_bf16(g, (const float*)Zu, rows, in.N, (const __hip_bfloat16*)pl.bf.V, ldr, cols, B, nullptr,
                               (float*)pl.bf.T, ldr, g_force_choice, st);
      return launch_cov_stencil(prec, g, Zu, rows, in.N, pl.bf.V, ldr, cols, B, nullptr, pl.bf.T, ldr, g_force_choice,
                                st);
    };
    bool seen[kTuneBuckets] = {false, false, false};
    for (int64_t div : {1, 4, 16}) {
      const int64_t B = std::min<int64_t>(cols, std::max<int64_t>(16, round_up(S / div, 16)));
      const int bucket = tune_bucket(B);
      if (seen[bucket]) continue;
      seen[bucket] = true;
      int best = 0;
      float best_ms = 0.f;
      for (int c : cands) {
        g_force_choice = c;
        hipError_t e = launch(B);  // warm-up (also sets kernel attributes)
        for (int r = 0; r < 5 && e == hipSuccess; ++r) {
          if (r == 1) e = hipEventRecord(e0, st);
          if (e == hipSuccess) e = launch(B);
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        g_force_choice = 0;
        if (e == hipErrorInvalidValue) {
          (void)hipGetLastError();  // a candidate that does not fit: skip it
          continue;
        }
        IE_HIP(e);
        float ms = 0.f;
        IE_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms /= 4.f;
        if (best == 0 || ms < best_ms) {
          best = c;
          best_ms = ms;
        }
      }
      if (best) set_tuned(key, bucket, best);
      if (report && rep < 2 * kTuneBuckets) {
        report[4 * rep + 0] = (int32_t)prec;
        report[4 * rep + 1] = (int32_t)B;
        report[4 * rep + 2] = best;
        report[4 * rep + 3] = (int32_t)(best_ms * 1000.f);  // microseconds per launch
        ++rep;
      }
    }
  }
  return INFOESRF_OK;
}

void infoesrf_autotune_reset(void) { tune_reset(); }

int infoesrf_warmstart_pairs(const infoesrf_problem* prob, int32_t Q, const double* s_nodes,
                             const double* p_weights, const double* y, float* X, float* cq, float* T,
                             const infoesrf_opts* opts, infoesrf_stats* stats, void* ws, size_t ws_bytes,
                             void* stream) {
  clear_error();
  IE_CHECK(X && cq && T, INFOESRF_ERR_INVALID_ARG, "X, cq and T must be non-NULL");
  IE_CHECK(!opts || opts->warm_start == INFOESRF_START_ZERO, INFOESRF_ERR_INVALID_ARG,
           "training pairs are solved from the zero start");
  Plan pl;
  Options op;
  hipStream_t st = static_cast<hipStream_t>(stream);
  IE_TRY(perturbation_solve(prob, Q, s_nodes, p_weights, y, opts, pl, op, ws, ws_bytes, st));
  Inst& in = pl.in;
  Sys& sy = pl.sy;
  hipLaunchKernelGGL(k_member_features, dim3(nb(in.N * in.m)), dim3(256), 0, st, sy.b, sy.ldm, sy.bnorm, in.m, in.N,
                     X);
  IE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_net_targets, dim3(nb(std::max<int64_t>(sy.S * in.m, Q))), dim3(256), 0, st, sy.u, sy.ldm,
                     sy.bnorm, sy.sigma, in.m, in.N, Q, cq, T);
  IE_HIP(hipGetLastError());
  return finish_status(pl, op, stats, 2 * pl.pr.k, st);
}

int infoesrf_batched_one_launch(const infoesrf_problem* probs, int32_t count, const int32_t* Q,
                                const infoesrf_opts* opts, const infoesrf_lattice* lattices) {
  clear_error();
  if (!probs || !Q || count < 1) return 0;
  infoesrf_opts o;
  if (opts) o = *opts;
  else infoesrf_default_opts(&o);
  if (o.apply_domain == INFOESRF_DOMAIN_OBS_LATTICE && !lattices) return 0;
  std::vector<infoesrf_opts> oj(count, o);
  if (o.apply_domain == INFOESRF_DOMAIN_OBS_LATTICE)
    for (int j = 0; j < count; ++j) oj[j].lattice = lattices[j];
  return batch_one_launch(probs, count, Q, oj) ? 1 : 0;
}

size_t infoesrf_batched_workspace_bytes(const infoesrf_problem* probs, int32_t count, const int32_t* Q,
                                        const infoesrf_opts* opts, const infoesrf_lattice* lattices) {
  clear_error();
  if (!probs || !Q || count < 1) {
    set_error("probs/Q must be non-NULL and count >= 1");
    return 0;
  }
  infoesrf_opts o;
  if (opts) o = *opts;
  else infoesrf_default_opts(&o);
  if (o.apply_domain == INFOESRF_DOMAIN_OBS_LATTICE && !lattices) {
    set_error("the observed-lattice domain needs lattices[count]");
    return 0;
  }
  std::vector<infoesrf_opts> oj(count, o);
  if (o.apply_domain == INFOESRF_DOMAIN_OBS_LATTICE)
    for (int j = 0; j < count; ++j) oj[j].lattice = lattices[j];
  const bool one = batch_one_launch(probs, count, Q, oj);
  size_t total = 0;
  int64_t systems = 0;
  for (int j = 0; j < count; ++j) {
    const size_t b = one ? combined_ws_bytes(&probs[j], Q[j], &oj[j]) : instance_ws_bytes(&probs[j], Q[j], true, &oj[j]);
    if (b == 0) {
      set_error("instance " + std::to_string(j) + ": " + g_last_error);
      return 0;
    }
    total += (b + 255) / 256 * 256;
    systems += (int64_t)Q[j] * probs[j].N + 1;
  }
  // two counter blocks per instance (perturbation and mean), and for one launch the batch arrays
  total += (size_t)2 * count * INFOESRF_NUM_COUNTERS * sizeof(int64_t) + 256;
  if (one) total += batch_area(nullptr, count, systems).bytes;
  return total;
}

int infoesrf_update_batched(const infoesrf_problem* probs, int32_t count, const int32_t* Q,
                            const double* const* s_nodes, const double* const* p_weights, const double* const* y,
                            double* const* mean_a, double* const* Xa_pert, const infoesrf_opts* opts,
                            const infoesrf_lattice* lattices, infoesrf_stats* stats, void* ws, size_t ws_bytes,
                            void* stream) {
  clear_error();
  IE_CHECK(probs && Q && s_nodes && p_weights && Xa_pert && count >= 1, INFOESRF_ERR_INVALID_ARG,
           "probs, Q, s_nodes, p_weights, Xa_pert must be non-NULL and count >= 1");
  IE_CHECK(ws != nullptr, INFOESRF_ERR_WORKSPACE, "workspace is NULL");
  infoesrf_opts o;
  if (opts) o = *opts;
  else infoesrf_default_opts(&o);
  const bool per_lattice = o.apply_domain == INFOESRF_DOMAIN_OBS_LATTICE;
  IE_CHECK(!per_lattice || lattices, INFOESRF_ERR_INVALID_ARG, "the observed-lattice domain needs lattices[count]");
  std::vector<infoesrf_opts> oj(count, o);
  if (per_lattice)
    for (int j = 0; j < count; ++j) oj[j].lattice = lattices[j];
  // every instance's systems in one persistent launch per sweep when each can run there;
  // otherwise a call per instance over a pool of streams, where the persistent kernel by default
  // only finishes each instance's last 64 systems (concurrent instances share the GPU)
  for (int j = 0; j < count; ++j) {
    const bool want_mean = mean_a && mean_a[j];
    IE_CHECK(!want_mean || (y && y[j]), INFOESRF_ERR_INVALID_ARG,
             "instance " + std::to_string(j) + ": the mean update needs y");
    IE_CHECK(Xa_pert[j] && s_nodes[j] && p_weights[j], INFOESRF_ERR_INVALID_ARG,
             "instance " + std::to_string(j) + ": s_nodes, p_weights and Xa_pert must be non-NULL");
  }
  const bool one = batch_one_launch(probs, count, Q, oj);
  if (!one && o.tail_systems == 0)
    for (int j = 0; j < count; ++j) oj[j].tail_systems = 64;
  // per-instance workspace slices and system offsets (validates every instance first)
  std::vector<size_t> off(count + 1, 0);
  std::vector<int64_t> sys_off(count + 1, 0);
  for (int j = 0; j < count; ++j) {
    const bool want_mean = mean_a && mean_a[j];
    const size_t b = one ? combined_ws_bytes(&probs[j], Q[j], &oj[j]) : instance_ws_bytes(&probs[j], Q[j], want_mean, &oj[j]);
    if (b == 0) {
      set_error("instance " + std::to_string(j) + ": " + g_last_error);
      return INFOESRF_ERR_INVALID_ARG;
    }
    off[j + 1] = off[j] + (b + 255) / 256 * 256;
    sys_off[j + 1] = sys_off[j] + (int64_t)Q[j] * probs[j].N + 1;
  }
  const size_t cnt_bytes = (size_t)2 * count * INFOESRF_NUM_COUNTERS * sizeof(int64_t);
  const size_t area = one ? batch_area(nullptr, count, sys_off[count]).bytes : 0;
  const size_t need = off[count] + cnt_bytes + area + 256;
  IE_CHECK(ws_bytes >= need, INFOESRF_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  char* base = static_cast<char*>(ws);
  int64_t* cnt = reinterpret_cast<int64_t*>(base + off[count]);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0;
  IE_HIP(hipGetDevice(&dev));
  // blocks of instances that fail before launching anything, or skip the mean, must read zero
  IE_HIP(launch_fill_i32(reinterpret_cast<int32_t*>(cnt), 0, (int64_t)4 * count * INFOESRF_NUM_COUNTERS, st));

  // largest instances first: cost ~ systems x observations x members x stencil width
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int j) {
    const infoesrf_problem& P = probs[j];
    return (double)Q[j] * P.N * (double)P.m * P.N * (2.0 * P.loc.bx + 1) * (2.0 * P.loc.bz + 1);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
  if (one) {
    const BatchArea ba = batch_area(base + off[count] + cnt_bytes, count, sys_off[count]);
    return batched_one_launch(probs, count, Q, s_nodes, p_weights, y, mean_a, Xa_pert, oj, stats, base, off, sys_off,
                              cnt, ba, order, o.host_sync != 0, st);
  }

  hipEvent_t fork = nullptr;
  IE_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
  std::vector<hipEvent_t> done(count, nullptr);
  std::vector<int> codes(count, 0);
  std::vector<std::string> msgs(count);
  auto cleanup = [&] {
    for (auto e : done)
      if (e) (void)hipEventDestroy(e);
    (void)hipEventDestroy(fork);
  };
  for (int j = 0; j < count; ++j) {
    if (hipEventCreateWithFlags(&done[j], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      set_error("hipEventCreate failed");
      return INFOESRF_ERR_HIP;
    }
  }
  if (hipEventRecord(fork, st) != hipSuccess) {
    cleanup();
    set_error("hipEventRecord failed");
    return INFOESRF_ERR_HIP;
  }

  // one instance: mean update (optional) then perturbation update, on stream ss
  auto run_one = [&](int j, hipStream_t ss) {
    int code = 0;
    if (hipStreamWaitEvent(ss, fork, 0) != hipSuccess) {
      codes[j] = INFOESRF_ERR_HIP;
      msgs[j] = "hipStreamWaitEvent failed";
      return;
    }
    void* wsj = base + off[j];
    const size_t wsb = off[j + 1] - off[j];
    infoesrf_stats sj{};
    const int64_t S = (int64_t)Q[j] * probs[j].N;
    if (stats) {
      sj.iters = stats->iters ? stats->iters + sys_off[j] : nullptr;
      sj.relres = stats->relres ? stats->relres + sys_off[j] : nullptr;
      sj.converged = stats->converged ? stats->converged + sys_off[j] : nullptr;
    }
    sj.counters = cnt + (int64_t)(2 * j) * INFOESRF_NUM_COUNTERS;
    code = infoesrf_perturbation_update(&probs[j], Q[j], s_nodes[j], p_weights[j], y ? y[j] : nullptr, Xa_pert[j],
                                        &oj[j], &sj, wsj, wsb, ss);
    if (code >= 0 && mean_a && mean_a[j]) {
      infoesrf_stats sm{};
      if (stats) {
        sm.iters = stats->iters ? stats->iters + sys_off[j] + S : nullptr;
        sm.relres = stats->relres ? stats->relres + sys_off[j] + S : nullptr;
        sm.converged = stats->converged ? stats->converged + sys_off[j] + S : nullptr;
      }
      sm.counters = cnt + (int64_t)(2 * j + 1) * INFOESRF_NUM_COUNTERS;
      const int cm = infoesrf_mean_update(&probs[j], y[j], mean_a[j], &oj[j], &sm, wsj, wsb, ss);
      code = (cm < 0) ? cm : std::max(code, cm);
    }
    codes[j] = code;
    if (code < 0) msgs[j] = g_last_error;
    if (hipEventRecord(done[j], ss) != hipSuccess && codes[j] >= 0) {
      codes[j] = INFOESRF_ERR_HIP;
      msgs[j] = "hipEventRecord failed";
    }
  };

  if (o.host_sync) {
    // every worker takes the next-largest instance from a shared cursor
    std::atomic<int> cursor{0};
    std::vector<std::function<void()>> tasks;
    const int nw = std::min<int>(WorkerPool::kWorkers, count);
    for (int w = 0; w < nw; ++w)
      tasks.emplace_back([&, dev] {
        hipStream_t ss = nullptr;
        hipError_t e = hipSetDevice(dev);
        if (e == hipSuccess) e = WorkerPool::worker_stream(dev, 0, &ss);
        for (int k = cursor.fetch_add(1); k < count; k = cursor.fetch_add(1)) {
          const int j = order[k];
          if (e != hipSuccess) {
            codes[j] = INFOESRF_ERR_HIP;
            msgs[j] = "worker device or stream set-up failed";
            (void)hipEventRecord(done[j], st);  // nothing ran: the join must not wait on it
            continue;
          }
          run_one(j, ss);
        }
      });
    WorkerPool::get().run(tasks);
  } else {
    // no host synchronization: every launch is issued from this thread, over this thread's
    // kWorkers streams in turn, so the call returns as soon as the work is enqueued
    for (int k = 0; k < count; ++k) {
      const int j = order[k];
      hipStream_t ss = nullptr;
      if (WorkerPool::worker_stream(dev, k % WorkerPool::kWorkers, &ss) != hipSuccess) {
        codes[j] = INFOESRF_ERR_HIP;
        msgs[j] = "stream creation failed";
        (void)hipEventRecord(done[j], st);
        continue;
      }
      run_one(j, ss);
    }
  }
  int worst_err = 0, worst_warn = 0, first_bad = -1;
  for (int j = 0; j < count; ++j) {
    if (codes[j] < worst_err) {
      worst_err = codes[j];
      first_bad = j;
    }
    worst_warn = std::max(worst_warn, codes[j]);
  }
  // join: the caller's stream waits for every instance
  for (int j = 0; j < count; ++j) {
    if (hipStreamWaitEvent(st, done[j], 0) != hipSuccess) {
      cleanup();
      set_error("hipStreamWaitEvent failed");
      return INFOESRF_ERR_HIP;
    }
  }
  if (stats && stats->counters) {
    hipLaunchKernelGGL(k_sum_counters, dim3(1), dim3(64), 0, st, cnt, 2 * count, stats->counters);
    if (hipGetLastError() != hipSuccess) {
      cleanup();
      set_error("counter reduction launch failed");
      return INFOESRF_ERR_HIP;
    }
  }
  cleanup();
  if (worst_err < 0) {
    set_error("instance " + std::to_string(first_bad) + ": " + msgs[first_bad]);
    return worst_err;
  }
  return worst_warn;
}

}  // extern "C"

namespace infoesrf {
namespace {
size_t instance_ws_bytes(const infoesrf_problem* P, int32_t Q, bool mean, const infoesrf_opts* opts) {
  const size_t bp = infoesrf_workspace_bytes(P, Q, opts);
  if (bp == 0) return 0;
  if (!mean) return bp;
  const size_t bm = infoesrf_workspace_bytes(P, 0, opts);
  if (bm == 0) return 0;
  return std::max(bp, bm);
}
}  // namespace
}  // namespace infoesrf
