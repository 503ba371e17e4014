// Block PCG over the members (the second alternative named in Sec. 3.2; O'Leary's method): for
// each node q the N systems ((1 + s_q) I + S) u_i = b_i are solved together, every column's
// iterate being the A-norm-optimal point of the sum of all columns' preconditioned Krylov
// spaces.  The node's limited-memory preconditioner (Appendix E) applies column by column.
//
// One iteration, for all live nodes at once, after the batched apply W = C_q P:
//   partials:  per 64-row chunk, P^T W, P^T R, W^T R, W^T W (N x N) and Phi^T W, Phi^T R,
//              (S Phi)^T W, (S Phi)^T R (p x N), diag R^T R;
//   reduce:    chunk sums in a fixed order;
//   small:     one workgroup per node: stop test on ||r_j||; G = P^T W = L L^T (Cholesky with
//              dependent directions dropped); A = G^+ P^T R; from the one-step updates
//              Phi^T R' = Phi^T R - (Phi^T W) A (the same for S Phi) the preconditioner's
//              coefficients c1, gamma of every column of R' = R - W A; W^T Z' with
//              Z' = R' - S Phi c1 - Phi gamma; B = G^+ W^T Z';
//   update:    X += P A, R = R - W A, P = Z' - P B, row by row (the new block is
//              A-orthogonal to the old one: the block CG short recurrence).
// Iteration 0 forms P = Z = M R from the right-hand sides.
#include <atomic>

#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kBcgChunk = 64;   // rows per partial
constexpr int kBcgSub = 32;     // rows staged in LDS at a time
constexpr int kBcgMaxN = 64;
constexpr int kBcgMaxP = 20;

// Offsets of the partial/reduced record of one node (N columns, p Ritz pairs).
struct BcgLayout {
  int64_t N, p;
  __host__ __device__ int64_t pw() const { return 0; }
  __host__ __device__ int64_t pr() const { return N * N; }
  __host__ __device__ int64_t wr() const { return 2 * N * N; }
  __host__ __device__ int64_t ww() const { return 3 * N * N; }
  __host__ __device__ int64_t fw() const { return 4 * N * N; }          // Phi^T W   (p x N, row a)
  __host__ __device__ int64_t fr() const { return 4 * N * N + p * N; }  // Phi^T R
  __host__ __device__ int64_t sw() const { return 4 * N * N + 2 * p * N; }
  __host__ __device__ int64_t sr() const { return 4 * N * N + 3 * p * N; }
  __host__ __device__ int64_t nr() const { return 4 * N * N + 4 * p * N; }  // diag R^T R (N)
  __host__ __device__ int64_t size() const { return 4 * N * N + 4 * p * N + N; }
  // coefficient record: A (N x N), B (N x N), c1 (p x N), gamma (p x N); row index first
  __host__ __device__ int64_t csize() const { return 2 * N * N + 2 * p * N; }
};

// kinds 0..3: the N x N products P^T W, P^T R, W^T R, W^T W; kind 4: the Ritz products and
// diag R^T R.  Grid (chunks, nodes, 5).  out[a * N + b] = sum_rows U[:, a] V[:, b].
__global__ __launch_bounds__(256) void k_bcg_partials(BcgState st, int with_w) {
  __shared__ double su[kBcgSub][kBcgMaxN + 4];  // columns padded to the 4-wide tiles
  __shared__ double sv[kBcgSub][kBcgMaxN + 4];
  __shared__ double sphi[kBcgSub][kBcgMaxP];
  __shared__ double ssphi[kBcgSub][kBcgMaxP];
  const int ch = blockIdx.x, q = blockIdx.y, kind = blockIdx.z;
  if (st.bdone[q] != 0) return;
  if (!with_w && kind < 4) return;
  const int tid = threadIdx.x;
  const int64_t N = st.N, m = st.m, ld = st.ld;
  const int p = st.p;
  const BcgLayout L{N, p};
  const int64_t col0 = (int64_t)q * N;
  double* out = st.part + ((int64_t)q * st.nch + ch) * L.size();
  const int64_t r0 = (int64_t)ch * kBcgChunk;
  const int64_t r1 = min<int64_t>(m, r0 + kBcgChunk);
  if (kind < 4) {
    // 4 x 4 output tiles per thread: thread t owns rows 4 (t / nt) .. +3 and columns 4 (t % nt) .. +3
    const double* U = (kind <= 1) ? st.P : st.W;
    const double* V = (kind == 0 || kind == 3) ? st.W : st.R;
    const int64_t off = kind == 0 ? L.pw() : (kind == 1 ? L.pr() : (kind == 2 ? L.wr() : L.ww()));
    const int nt = (int)((N + 3) / 4);
    const int ta = tid / nt, tb = tid % nt;
    const bool act = ta < nt;
    double acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
    for (int64_t s0 = r0; s0 < r1; s0 += kBcgSub) {
      const int rows = (int)min<int64_t>(kBcgSub, r1 - s0);
      __syncthreads();
      for (int o = tid; o < kBcgSub * kBcgMaxN; o += 256) {
        const int c = o / kBcgSub, rr = o % kBcgSub;
        const bool ok = rr < rows && c < N;
        su[rr][c] = ok ? U[(col0 + c) * ld + s0 + rr] : 0.0;
        sv[rr][c] = ok ? V[(col0 + c) * ld + s0 + rr] : 0.0;
      }
      __syncthreads();
      if (act) {
        for (int rr = 0; rr < kBcgSub; ++rr) {
          double u[4], v[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            u[x] = su[rr][4 * ta + x];
            v[x] = sv[rr][4 * tb + x];
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] += u[x] * v[y];
        }
      }
    }
    if (act) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          const int a = 4 * ta + x, b = 4 * tb + y;
          if (a < N && b < N) out[off + a * N + b] = acc[x][y];
        }
    }
    return;
  }
  // kind 4: Phi^T W, Phi^T R, (S Phi)^T W, (S Phi)^T R and diag R^T R
  const int64_t nout = 4 * (int64_t)p * N + N;
  double acc[24];
#pragma unroll
  for (int e = 0; e < 24; ++e) acc[e] = 0.0;
  for (int64_t s0 = r0; s0 < r1; s0 += kBcgSub) {
    const int rows = (int)min<int64_t>(kBcgSub, r1 - s0);
    __syncthreads();
    for (int o = tid; o < kBcgSub * N; o += 256) {
      const int c = o / kBcgSub, rr = o % kBcgSub;
      const bool ok = rr < rows;
      su[rr][c] = (ok && with_w) ? st.W[(col0 + c) * ld + s0 + rr] : 0.0;
      sv[rr][c] = ok ? st.R[(col0 + c) * ld + s0 + rr] : 0.0;
    }
    for (int o = tid; o < kBcgSub * p; o += 256) {
      const int a = o / kBcgSub, rr = o % kBcgSub;
      const bool ok = rr < rows;
      sphi[rr][a] = ok ? st.Phi[a * st.ldphi + s0 + rr] : 0.0;
      ssphi[rr][a] = ok ? st.SPhi[a * st.ldphi + s0 + rr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 24; ++e) {
      const int64_t o = tid + 256 * e;
      if (o < nout) {
        double t = 0.0;
        if (o < 4 * (int64_t)p * N) {
          const int fam = (int)(o / (p * N));
          const int64_t w = o % (p * N);
          const int a = (int)(w / N), b = (int)(w % N);
          const bool ritz_s = fam >= 2;            // S Phi rows
          const bool against_r = (fam & 1) != 0;   // R columns
          for (int rr = 0; rr < kBcgSub; ++rr) {
            const double f = ritz_s ? ssphi[rr][a] : sphi[rr][a];
            t += f * (against_r ? sv[rr][b] : su[rr][b]);
          }
        } else {
          const int b = (int)(o - 4 * (int64_t)p * N);
          for (int rr = 0; rr < kBcgSub; ++rr) t += sv[rr][b] * sv[rr][b];
        }
        acc[e] += t;
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 24; ++e) {
    const int64_t o = tid + 256 * e;
    if (o < nout) out[L.fw() + o] = acc[e];
  }
}

// red[q][e] = sum over chunks of part[q][ch][e] (chunks in order).  Grid (ceil(size/256), nodes).
__global__ void k_bcg_reduce(BcgState st) {
  const int q = blockIdx.y;
  if (st.bdone[q] != 0) return;
  const BcgLayout L{st.N, st.p};
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= L.size()) return;
  const double* src = st.part + (int64_t)q * st.nch * L.size() + e;
  double a = 0.0;
  for (int c = 0; c < st.nch; ++c) a += src[(int64_t)c * L.size()];
  st.red[(int64_t)q * L.size() + e] = a;
}

constexpr int kSmallThreads = 1024;  // 16 wavefronts: the per-node chains hide each other's latency
constexpr int kSmallPer = (kBcgMaxP * kBcgMaxN + kSmallThreads - 1) / kSmallThreads;

// sum_l x[l] y[l * stride] with four independent partial sums (x in LDS or L2, y in LDS).
__device__ inline double dot_rows(const double* x, const double* y, int n, int stride) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int l = 0;
  for (; l + 4 <= n; l += 4) {
    s0 += x[l] * y[l * stride];
    s1 += x[l + 1] * y[(l + 1) * stride];
    s2 += x[l + 2] * y[(l + 2) * stride];
    s3 += x[l + 3] * y[(l + 3) * stride];
  }
  for (; l < n; ++l) s0 += x[l] * y[l * stride];
  return (s0 + s1) + (s2 + s3);
}

// One workgroup per node.  mode 0: iteration 0 (coefficients of P = M R); mode 1: iteration `it`.
// LDS (dynamic, bcg_small_lds doubles): the inverse of G, A, a work matrix, Phi^T W and
// (S Phi)^T W, c1 and gamma.  G is inverted by symmetric sweeps (Gauss-Jordan on an SPD matrix,
// all N^2 entries per step in parallel).  An index whose pivot (the energy of its column outside
// the span of the columns kept before it) is below 1e-9 of the column's own energy, or below
// 1e-12 of the largest diagonal entry, is taken as dependent and left out (its row and column of
// the inverse are 0).  The block is rank-deficient from the start: the members' perturbations
// sum to zero, and so do their right-hand sides.
__global__ __launch_bounds__(kSmallThreads) void k_bcg_small(BcgState st, int mode, int it, int ww_fits) {
  extern __shared__ double lds[];
  __shared__ double srow[kBcgMaxN], scol[kBcgMaxN], sdiag[kBcgMaxN];
  __shared__ int keep[kBcgMaxN];
  __shared__ int s_state;
  __shared__ double s_dmax;
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  if (st.bdone[q] != 0) return;
  const int N = (int)st.N, p = st.p;
  const int NN = N * N, PN = p * N;
  const BcgLayout L{st.N, p};
  const double* rd = st.red + (int64_t)q * L.size();
  double* cf = st.coef + (int64_t)q * L.csize();
  double* Mi = lds;            // N x N: G, then -G^+ after the sweeps
  double* A = Mi + NN;         // N x N
  double* T = A + NN;          // N x N work
  double* FW = T + NN;         // p x N Phi^T W
  double* SW = FW + PN;        // p x N (S Phi)^T W
  double* C1 = SW + PN;        // p x N
  double* GA = C1 + PN;        // p x N
  double* WW = GA + PN;        // N x N W^T W when the LDS holds it (ww_lds), else read from L2
  const int64_t col0 = (int64_t)q * N;
  const double sig1 = 1.0 + st.sigma[col0];
  const bool ww_lds = ww_fits;
  // stop test on the current residual block
  if (tid == 0) s_state = 0;
  __syncthreads();
  for (int j = tid; j < N; j += kSmallThreads) {
    const double nrm = sqrt(fmax(rd[L.nr() + j], 0.0));
    const double bn = st.bnorm[col0 + j];
    st.relres[col0 + j] = bn > 0.0 ? nrm / bn : 0.0;
    if (!(nrm <= st.thresh[col0 + j])) atomicOr(&s_state, 1);  // some column is still live
  }
  __syncthreads();
  int state = 0;
  if (s_state == 0) state = 1;
  else if (mode == 1 && it > st.max_iter) state = 2;
  if (state != 0) {
    for (int j = tid; j < N; j += kSmallThreads) {
      const double nrm = sqrt(fmax(rd[L.nr() + j], 0.0));
      st.done[col0 + j] = (nrm <= st.thresh[col0 + j]) ? 1 : 2;
    }
    if (tid == 0) st.bdone[q] = state;
    return;
  }
  for (int j = tid; j < N; j += kSmallThreads) st.iters[col0 + j] = mode == 1 ? it : 0;
  for (int o = tid; o < PN; o += kSmallThreads) {
    FW[o] = mode == 1 ? rd[L.fw() + o] : 0.0;
    SW[o] = mode == 1 ? rd[L.sw() + o] : 0.0;
  }
  if (mode == 1) {
    for (int o = tid; o < NN; o += kSmallThreads) {
      const int a = o / N, b = o % N;
      Mi[o] = 0.5 * (rd[L.pw() + a * N + b] + rd[L.pw() + b * N + a]);
      T[o] = rd[L.pr() + o];
    }
    __syncthreads();
    if (tid == 0) {
      double dmax = 0.0;
      for (int a = 0; a < N; ++a) dmax = fmax(dmax, Mi[a * N + a]);
      s_dmax = dmax;
      if (!(dmax > 0.0) || !isfinite(dmax)) atomicOr(st.flags, isfinite(dmax) ? kFlagNotSPD : kFlagNumeric);
    }
    __syncthreads();
    if (tid < N) sdiag[tid] = Mi[tid * N + tid];
    __syncthreads();
    const double tol = 1e-12 * s_dmax;
    for (int a = 0; a < N; ++a) {
      // pivot = the part of column a's energy outside the span of the columns kept before it
      const double d = Mi[a * N + a];
      const bool piv = d > tol && d > 1e-9 * sdiag[a];  // the same value in every thread
      if (tid < N) {
        srow[tid] = Mi[a * N + tid];
        scol[tid] = Mi[tid * N + a];
      }
      if (tid == 0) keep[a] = piv;
      __syncthreads();
      if (piv) {
        const double di = 1.0 / d;
        for (int o = tid; o < NN; o += kSmallThreads) {
          const int i = o / N, j = o % N;
          double v;
          if (i == a && j == a) v = -di;
          else if (i == a) v = srow[j] * di;
          else if (j == a) v = scol[i] * di;
          else v = Mi[o] - scol[i] * srow[j] * di;
          Mi[o] = v;
        }
      }
      __syncthreads();
    }
    // A = G^+ (P^T R) = -Mi T restricted to the kept indices (Mi's dropped rows and columns are
    // zeroed first, so the products need no test)
    for (int o = tid; o < NN; o += kSmallThreads) {
      const int a = o / N, l = o % N;
      if (!keep[a] || !keep[l]) Mi[o] = 0.0;
    }
    __syncthreads();
    for (int o = tid; o < NN; o += kSmallThreads) A[o] = -dot_rows(Mi + (o / N) * N, T + (o % N), N, N);
    if (ww_lds)
      for (int o = tid; o < NN; o += kSmallThreads) WW[o] = rd[L.ww() + o];
    __syncthreads();
  }
  // Ritz dots of the new residual R' = R - W A (kept in registers), the coefficients c1
  double d1r[kSmallPer], d2r[kSmallPer];
#pragma unroll
  for (int e = 0; e < kSmallPer; ++e) {
    const int o = tid + kSmallThreads * e;
    d1r[e] = 0.0;
    d2r[e] = 0.0;
    if (o < PN) {
      const int a = o / N, j = o % N;
      double d1 = rd[L.fr() + o], d2 = rd[L.sr() + o];
      if (mode == 1) {
        d1 -= dot_rows(FW + a * N, A + j, N, N);
        d2 -= dot_rows(SW + a * N, A + j, N, N);
      }
      d1r[e] = d1;
      d2r[e] = d2;
      C1[o] = d1 / (sig1 + st.theta[a]);
    }
  }
  __syncthreads();
  const double beta_l = sig1 + *st.dmin;
#pragma unroll
  for (int e = 0; e < kSmallPer; ++e) {
    const int o = tid + kSmallThreads * e;
    if (o < PN) {
      const int a = o / N, j = o % N;
      const double* Gpp = st.G;
      const double* Gps = st.G + p * p;
      const double* Gss = st.G + 2 * p * p;
      double mc = 0.0;
      for (int l = 0; l < p; ++l)
        mc += (Gss[a * p + l] + sig1 * (Gps[a * p + l] + Gps[l * p + a]) + sig1 * sig1 * Gpp[a * p + l]) *
              C1[l * N + j];
      const double c2 = (d2r[e] + sig1 * d1r[e] - mc) / (sig1 + st.theta[a]);
      GA[o] = (sig1 - beta_l) * C1[o] + c2;
    }
  }
  __syncthreads();
  if (mode == 1) {
    // W^T Z' = (W^T R - W^T W A) - (W^T S Phi) c1 - (W^T Phi) gamma into T, then B = G^+ W^T Z'
    for (int o = tid; o < NN; o += kSmallThreads) {
      const int a = o / N, j = o % N;
      const double* ww = (ww_lds ? WW : rd + L.ww()) + a * N;
      double v = rd[L.wr() + o] - dot_rows(ww, A + j, N, N);
      for (int t = 0; t < p; ++t) v -= SW[t * N + a] * C1[t * N + j] + FW[t * N + a] * GA[t * N + j];
      T[o] = v;
    }
    __syncthreads();
    for (int o = tid; o < NN; o += kSmallThreads) {
      cf[NN + o] = -dot_rows(Mi + (o / N) * N, T + (o % N), N, N);  // B
      cf[o] = A[o];
    }
  } else {
    for (int o = tid; o < NN; o += kSmallThreads) {
      cf[o] = 0.0;
      cf[NN + o] = 0.0;
    }
  }
  for (int o = tid; o < PN; o += kSmallThreads) {
    cf[2 * NN + o] = C1[o];
    cf[2 * NN + PN + o] = GA[o];
  }
}

// Row-wise update of node q's block: X += P A, R' = R - W A, P = (R' - S Phi c1 - Phi gamma) - P B.
// Grid (ceil(m / 32), nodes); 256 threads = 32 rows x 8 column groups (columns j = g, g + 8, ...).
// LDS (dynamic, bcg_update_lds doubles): the coefficient record and the block's rows of P and W
// (staged before P is overwritten).
__global__ __launch_bounds__(256) void k_bcg_update(BcgState st, int mode) {
  extern __shared__ double lds[];
  const int q = blockIdx.y;
  if (st.bdone[q] != 0) return;
  const int tid = threadIdx.x;
  const int rr = tid & 31, cg = tid >> 5;
  const int N = (int)st.N, p = st.p;
  const int NN = N * N, PN = p * N;
  const int64_t m = st.m, ld = st.ld;
  const int64_t r = (int64_t)blockIdx.x * 32 + rr;
  const int64_t col0 = (int64_t)q * N;
  const BcgLayout L{st.N, p};
  double* cA = lds;
  double* cB = cA + NN;
  double* cC1 = cB + NN;
  double* cGA = cC1 + PN;
  double* sp = cGA + PN;  // N x 32
  double* sw = sp + 32 * N;
  const double* cf = st.coef + (int64_t)q * L.csize();
  for (int o = tid; o < 2 * NN + 2 * PN; o += 256) lds[o] = cf[o];
  for (int o = tid; o < 32 * N; o += 256) {
    const int l = o / 32, k = o % 32;
    const int64_t rk = (int64_t)blockIdx.x * 32 + k;
    sp[o] = rk < m ? st.P[(col0 + l) * ld + rk] : 0.0;
    sw[o] = (rk < m && mode == 1) ? st.W[(col0 + l) * ld + rk] : 0.0;
  }
  __syncthreads();
  if (r >= m) return;
  constexpr int kJ = kBcgMaxN / 8;  // columns per thread
  double ax[kJ], aw[kJ], ab[kJ];
#pragma unroll
  for (int u = 0; u < kJ; ++u) {
    ax[u] = 0.0;
    aw[u] = 0.0;
    ab[u] = 0.0;
  }
  if (mode == 1) {
    for (int l = 0; l < N; ++l) {
      const double pl = sp[l * 32 + rr], wl = sw[l * 32 + rr];
#pragma unroll
      for (int u = 0; u < kJ; ++u) {
        const int j = cg + 8 * u;
        if (j < N) {
          const double a = cA[l * N + j], b = cB[l * N + j];
          ax[u] += pl * a;
          aw[u] += wl * a;
          ab[u] += pl * b;
        }
      }
    }
  }
  double ph[kBcgMaxP], sph[kBcgMaxP];
  for (int t = 0; t < p; ++t) {
    ph[t] = st.Phi[t * st.ldphi + r];
    sph[t] = st.SPhi[t * st.ldphi + r];
  }
#pragma unroll
  for (int u = 0; u < kJ; ++u) {
    const int j = cg + 8 * u;
    if (j < N) {
      const int64_t idx = (col0 + j) * ld + r;
      const double rn = st.R[idx] - aw[u];
      double z = rn;
      for (int t = 0; t < p; ++t) z -= sph[t] * cC1[t * N + j] + ph[t] * cGA[t * N + j];
      if (mode == 1) {
        st.X[idx] += ax[u];
        st.R[idx] = rn;
      }
      st.P[idx] = z - ab[u];
    }
  }
}

// act = the systems of the nodes still iterating (node-major), *nact their number (one block).
__global__ void k_bcg_list(const int32_t* bdone, int Q, int64_t N, int32_t* act, int32_t* nact) {
  __shared__ int32_t pre[kMaxQ + 1];
  if (threadIdx.x == 0) {
    int32_t c = 0;
    for (int q = 0; q < Q; ++q) {
      pre[q] = c;
      if (bdone[q] == 0) c += (int32_t)N;
    }
    pre[Q] = c;
    *nact = c;
  }
  __syncthreads();
  for (int64_t t = threadIdx.x; t < (int64_t)Q * N; t += blockDim.x) {
    const int q = (int)(t / N);
    if (bdone[q] == 0) act[pre[q] + (t - (int64_t)q * N)] = (int32_t)t;
  }
}

}  // namespace

hipError_t launch_bcg_iteration(const BcgState& s, int mode, int it, hipStream_t st) {
  if (s.N < 1 || s.N > kBcgMaxN || s.p < 0 || s.p > kBcgMaxP || s.Q < 1 || s.Q > kMaxQ) return hipErrorInvalidValue;
  if (s.nch != (int)((s.m + kBcgChunk - 1) / kBcgChunk)) return hipErrorInvalidValue;
  const BcgLayout L{s.N, s.p};
  hipLaunchKernelGGL(k_bcg_partials, dim3((unsigned)s.nch, (unsigned)s.Q, 5), dim3(256), 0, st, s, mode);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bcg_reduce, dim3((unsigned)((L.size() + 255) / 256), (unsigned)s.Q), dim3(256), 0, st, s);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t small_base = sizeof(double) * (size_t)(3 * s.N * s.N + 4 * s.p * s.N);
  const size_t small_ww = small_base + sizeof(double) * (size_t)(s.N * s.N);
  const int ww_fits = small_ww <= 140 * 1024;  // W^T W in LDS too
  const size_t small_lds = ww_fits ? small_ww : small_base;
  const size_t upd_lds = sizeof(double) * (size_t)(2 * s.N * s.N + 2 * s.p * s.N + 64 * s.N);
  static std::atomic<bool> attr{false};  // set once (before any graph capture that follows)
  if (!attr.load(std::memory_order_acquire)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bcg_small), hipFuncAttributeMaxDynamicSharedMemorySize,
                            150 * 1024);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_bcg_update), hipFuncAttributeMaxDynamicSharedMemorySize,
                            150 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
  }
  if (small_lds > 140 * 1024 || upd_lds > 140 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bcg_small, dim3((unsigned)s.Q), dim3(kSmallThreads), small_lds, st, s, mode, it, ww_fits);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bcg_update, dim3((unsigned)((s.m + 31) / 32), (unsigned)s.Q), dim3(256), upd_lds, st, s,
                     mode);
  return hipGetLastError();
}

hipError_t launch_bcg_list(const int32_t* bdone, int Q, int64_t N, int32_t* act, int32_t* nact, hipStream_t st) {
  if (Q < 1 || Q > kMaxQ) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_bcg_list, dim3(1), dim3(256), 0, st, bdone, Q, N, act, nact);
  return hipGetLastError();
}

int64_t bcg_partial_doubles(int64_t m, int64_t N, int p, int Q) {
  const BcgLayout L{N, p};
  return (int64_t)Q * ((m + kBcgChunk - 1) / kBcgChunk) * L.size();
}
int64_t bcg_reduced_doubles(int64_t N, int p, int Q) { return (int64_t)Q * BcgLayout{N, p}.size(); }
int64_t bcg_coef_doubles(int64_t N, int p, int Q) { return (int64_t)Q * BcgLayout{N, p}.csize(); }
int bcg_chunks(int64_t m) { return (int)((m + kBcgChunk - 1) / kBcgChunk); }

}  // namespace infoesrf
