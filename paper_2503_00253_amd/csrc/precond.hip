// Limited-memory preconditioner setup (Appendix E): Ritz pairs of S from a
// randomized symmetric eigendecomposition (Halko, Martinsson & Tropp: range
// finder followed by the direct eigendecomposition of the projected matrix).
//
//   Y = S Omega, Qb = orth(Y) (Cholesky-QR applied twice), T = Qb^T (S Qb),
//   T = V diag(lambda) V^T, Phi = Qb V_p, S Phi = (S Qb) V_p, theta = lambda_p.
//
// All small dense steps run on one workgroup so the setup needs no host round
// trip and can be captured in a HIP graph.
#include <atomic>

#include "internal.hpp"

namespace infoesrf {

namespace {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): counter-based generator.
__device__ inline void philox_round(uint32_t* c, const uint32_t* k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint64_t p0 = (uint64_t)M0 * c[0];
  const uint64_t p1 = (uint64_t)M1 * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

__device__ inline void philox4x32_10(uint32_t* c, uint32_t k0, uint32_t k1) {
  uint32_t k[2] = {k0, k1};
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
}

__global__ void k_sketch(uint64_t seed, int64_t m, int k, double* __restrict__ out, int64_t ld) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * k) return;
  uint32_t c[4] = {(uint32_t)t, (uint32_t)(t >> 32), 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  // two 53-bit uniforms in (0, 1], Box-Muller
  const double u1 = ((double)((((uint64_t)c[0]) << 21) ^ (uint64_t)(c[1] >> 11)) + 1.0) * 0x1p-53;
  const double u2 = ((double)((((uint64_t)c[2]) << 21) ^ (uint64_t)(c[3] >> 11)) + 0.5) * 0x1p-53;
  const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  const int64_t j = t / m, r = t % m;
  out[j * ld + r] = g;
}

// The sketch of k_sketch over all ld rows of its k columns (rows past m zero), with the list of
// the k columns as systems (act = 0 .. k-1, *nact = k) and their shifts (sig = -1: pure S).
__global__ void k_sketch_setup(uint64_t seed, int64_t m, int k, double* __restrict__ out, int64_t ld,
                               int32_t* __restrict__ act, int32_t* __restrict__ nact, double* __restrict__ sig,
                               int nsig) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < nsig) sig[t] = -1.0;
  if (t < k) act[t] = (int32_t)t;
  if (t == 0) *nact = k;
  if (t >= ld * k) return;
  const int64_t j = t / ld, r = t % ld;
  double g = 0.0;
  if (r < m) {
    const int64_t c = j * m + r;  // the counter of k_sketch's entry (r, j)
    uint32_t ctr[4] = {(uint32_t)c, (uint32_t)(c >> 32), 0u, 0u};
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u1 = ((double)((((uint64_t)ctr[0]) << 21) ^ (uint64_t)(ctr[1] >> 11)) + 1.0) * 0x1p-53;
    const double u2 = ((double)((((uint64_t)ctr[2]) << 21) ^ (uint64_t)(ctr[3] >> 11)) + 0.5) * 0x1p-53;
    g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
  out[t] = g;
}

// partial Gram over a chunk of kGramChunk rows: scratch[chunk][a*k+b].  The chunk's rows of A and
// B are staged in LDS first (unit-stride reads along each column), then each thread sums its
// entries from LDS.
constexpr int kGramChunk = 32;
__global__ __launch_bounds__(256) void k_gram_partial(Strided A, Strided B, int64_t m, int k,
                                                      double* __restrict__ scratch) {
  __shared__ double sa[kMaxSketch][kGramChunk + 1];
  __shared__ double sb[kMaxSketch][kGramChunk + 1];
  const int64_t r0 = blockIdx.x * (int64_t)kGramChunk;
  const int rows = (int)min<int64_t>(kGramChunk, m - r0);
  for (int o = threadIdx.x; o < k * kGramChunk; o += blockDim.x) {
    const int a = o / kGramChunk, r = o % kGramChunk;
    const bool ok = r < rows;
    sa[a][r] = ok ? A.ptr[(r0 + r) * A.rs + a * A.cs] : 0.0;
    sb[a][r] = ok ? B.ptr[(r0 + r) * B.rs + a * B.cs] : 0.0;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int a = t / k, b = t % k;
    double s0 = 0.0, s1 = 0.0;
    for (int r = 0; r < kGramChunk; r += 2) {
      s0 += sa[a][r] * sb[b][r];
      s1 += sa[a][r + 1] * sb[b][r + 1];
    }
    scratch[blockIdx.x * (int64_t)k * k + t] = s0 + s1;
  }
}

__global__ void k_gram_reduce(const double* __restrict__ scratch, int nchunks, int k, double* __restrict__ G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * k) return;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += scratch[(int64_t)c * k * k + t];
  G[t] = acc;
}

// A Cholesky pivot at or below this fraction of the largest diagonal entry of the Gram matrix
// marks a column that depends on the earlier ones (to rounding): Y = S Omega has rank at most
// rank(S), which falls below the sketch width when, e.g., L = 1 and N - 1 < p + oversample.
// Such a column gets a zero row in R and a zero column in Q; its Ritz value is then zero.
constexpr double kCholDrop = 1e-12;

// G (k x k, row-major, symmetric PSD) -> inverse of its upper Cholesky factor R (G = R^T R), in
// place, with dependent columns (pivot <= kCholDrop max diag G) given zero rows in R and zero
// columns in R^{-1}.  A non-finite pivot sets the numeric flag.  One wavefront; the inverse's
// columns are built in LDS.
__global__ void k_chol_inv(double* G, int k, int32_t* flags) {
  __shared__ double R[kMaxSketch * kMaxSketch];
  __shared__ double X[kMaxSketch * kMaxSketch];
  __shared__ int bad;
  __shared__ double gmax;
  const int t = threadIdx.x;
  if (t == 0) {
    bad = 0;
    double g = 0.0;
    for (int j = 0; j < k; ++j) g = fmax(g, G[j * k + j]);
    gmax = g;
  }
  for (int e = t; e < k * k; e += blockDim.x) R[e] = G[e];
  __syncthreads();
  // right-looking Cholesky, column j
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double d = R[j * k + j];
      if (!isfinite(d)) bad = 1;
      R[j * k + j] = (d > kCholDrop * gmax) ? sqrt(d) : 0.0;
    }
    __syncthreads();
    const double rjj = R[j * k + j];
    for (int c = j + 1 + t; c < k; c += blockDim.x) R[j * k + c] = rjj > 0.0 ? R[j * k + c] / rjj : 0.0;
    __syncthreads();
    for (int e = t; e < (k - j - 1) * (k - j - 1); e += blockDim.x) {
      const int a = j + 1 + e / (k - j - 1), b = j + 1 + e % (k - j - 1);
      if (b >= a) R[a * k + b] -= R[j * k + a] * R[j * k + b];
    }
    __syncthreads();
  }
  // R is upper triangular in R[a*k+b], b >= a.  Invert by columns: Rinv[:, c] solves R x = e_c
  // (X[a*k + c] = x_a, written by the thread of column c only); x_a = 0 on a dropped row.
  for (int c = t; c < k; c += blockDim.x) {
    for (int a = k - 1; a >= 0; --a) {
      double s = (a == c) ? 1.0 : 0.0;
      for (int b = a + 1; b < k; ++b) s -= R[a * k + b] * X[b * k + c];
      X[a * k + c] = (a <= c && R[a * k + a] > 0.0) ? s / R[a * k + a] : 0.0;
    }
  }
  __syncthreads();
  for (int e = t; e < k * k; e += blockDim.x) G[e] = X[e];
  if (t == 0 && bad) atomicOr(flags, kFlagNumeric);
}

// out(r, j) = sum_a A(r, a) M[a*kout + j]
__global__ void k_right_mult(Strided A, int64_t m, int k, const double* __restrict__ M, int kout,
                             double* __restrict__ out, int64_t ors, int64_t ocs) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= m * kout) return;
  const int64_t r = t % m;
  const int j = (int)(t / m);
  double acc = 0.0;
  for (int a = 0; a < k; ++a) acc += A.ptr[r * A.rs + a * A.cs] * M[a * kout + j];
  out[r * ors + j * ocs] = acc;
}

// Jacobi eigendecomposition of a small symmetric matrix on one workgroup with the round-robin
// (tournament) ordering: each step rotates k/2 disjoint index pairs at once, k-1 steps make a
// sweep in which every pair is visited once.  A step is two phases: the rotations of the pairs,
// then, with A double-buffered, every thread's 2 x 2 blocks of the next A = J^T A J (one block
// per pair of pairs) and its pair of eigenvector entries (V J, in place: each pair of entries
// has one owner).  T (k x k row-major) is read;
// evec[a*k + j] = component a of eigenvector j.
__device__ inline void jacobi_player(int slot, int step, int ke, int k, int* p, int* q, int t) {
  // players: slot 0 fixed, slots 1..ke-1 rotate by `step`; pair t holds slots t and ke-1-t
  auto player = [&](int sl) { return sl == 0 ? 0 : 1 + (sl - 1 + step) % (ke - 1); };
  int a = player(t), b = player(ke - 1 - t);
  if (a > b) {
    const int tmp = a;
    a = b;
    b = tmp;
  }
  *p = a;
  *q = b;
  (void)slot;
  (void)k;
}

// The rotation (c, s) that zeroes a_pq of the 2 x 2 block [a_pp a_pq; a_pq a_qq]: the smaller
// root t of t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 a_pq), written as
// t = sign(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)): one square root and one division.
__device__ inline void jacobi_cs(double app, double aqq, double apq, double* c, double* sn) {
  const double d = aqq - app;
  const double a2 = 2.0 * apq;
  const double tt = (d >= 0.0 ? a2 : -a2) / (fabs(d) + sqrt(d * d + a2 * a2));
  *c = rsqrt(1.0 + tt * tt);
  *sn = tt * *c;
}

__device__ inline void jacobi_rot(const double* A, int k, int p, int q, double* c, double* sn) {
  *c = 1.0;
  *sn = 0.0;
  if (q >= k) return;  // the dummy player of an odd k
  const double apq = A[p * k + q];
  if (apq == 0.0) return;
  jacobi_cs(A[p * k + p], A[q * k + q], apq, c, sn);
}

__global__ __launch_bounds__(256) void k_sym_eig(double* T, int k, double* evec, double* evals) {
  __shared__ double Ab[2][kMaxSketch * kMaxSketch];
  __shared__ double Vv[kMaxSketch * kMaxSketch];
  __shared__ double cs_c[kMaxSketch / 2], cs_s[kMaxSketch / 2];
  __shared__ int pp[kMaxSketch / 2], qq[kMaxSketch / 2];
  __shared__ double red[2][4];
  const int t = threadIdx.x;
  const int ke = k + (k & 1);  // even number of players; index k (if odd) is a dummy
  const int half = ke / 2;
  for (int e = t; e < k * k; e += blockDim.x) {
    Ab[0][e] = 0.5 * (T[e] + T[(e % k) * k + e / k]);
    Vv[e] = (e / k == e % k) ? 1.0 : 0.0;
  }
  __syncthreads();
  int cur = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    const double* A = Ab[cur];
    double off = 0.0, dia = 0.0;
    for (int e = t; e < k * k; e += blockDim.x) {
      const double v = A[e] * A[e];
      if (e / k == e % k) dia += v;
      else off += v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o, 64);
      dia += __shfl_xor(dia, o, 64);
    }
    if ((t & 63) == 0) {
      red[0][t >> 6] = off;
      red[1][t >> 6] = dia;
    }
    __syncthreads();
    const double toff = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    const double tdia = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    __syncthreads();
    // relative off-diagonal norm 1e-14 (FP64 Ritz vectors)
    if (toff <= 1e-28 * tdia) break;
    for (int step = 0; step < ke - 1; ++step) {
      const double* Ac = Ab[cur];
      double* An = Ab[cur ^ 1];
      if (t < half) {
        int p, q;
        jacobi_player(0, step, ke, k, &p, &q, t);
        double c, sn;
        jacobi_rot(Ac, k, p, q, &c, &sn);
        pp[t] = p;
        qq[t] = q;
        cs_c[t] = c;
        cs_s[t] = sn;
      }
      __syncthreads();
      // 2 x 2 blocks of J^T A J: pairs (i1, i2), one block per thread
      for (int w = t; w < half * half; w += blockDim.x) {
        const int i1 = w / half, i2 = w % half;
        const int p1 = pp[i1], q1 = qq[i1], p2 = pp[i2], q2 = qq[i2];
        const double c1 = cs_c[i1], s1 = cs_s[i1], c2 = cs_c[i2], s2 = cs_s[i2];
        const bool r1 = q1 < k, r2 = q2 < k;  // a dummy index has no row or column
        const double app = Ac[p1 * k + p2];
        const double apq = r2 ? Ac[p1 * k + q2] : 0.0;
        const double aqp = r1 ? Ac[q1 * k + p2] : 0.0;
        const double aqq = (r1 && r2) ? Ac[q1 * k + q2] : 0.0;
        // rows: [p1; q1] <- [c1 -s1; s1 c1] [p1; q1], then columns likewise with (c2, s2)
        const double xp = c1 * app - s1 * aqp, xq = s1 * app + c1 * aqp;  // column p2
        const double yp = c1 * apq - s1 * aqq, yq = s1 * apq + c1 * aqq;  // column q2
        An[p1 * k + p2] = c2 * xp - s2 * yp;
        if (r2) An[p1 * k + q2] = s2 * xp + c2 * yp;
        if (r1) An[q1 * k + p2] = c2 * xq - s2 * yq;
        if (r1 && r2) An[q1 * k + q2] = s2 * xq + c2 * yq;
      }
      // eigenvector columns p, q of every pair: row j, pair i, one owner each
      for (int w = t; w < half * k; w += blockDim.x) {
        const int i = w / k, j = w % k;
        const double sn = cs_s[i];
        if (sn == 0.0) continue;
        const int pq = pp[i], q2 = qq[i];
        const double c = cs_c[i];
        const double vp = Vv[j * k + pq], vq = Vv[j * k + q2];
        Vv[j * k + pq] = c * vp - sn * vq;
        Vv[j * k + q2] = sn * vp + c * vq;
      }
      __syncthreads();
      cur ^= 1;
    }
  }
  const double* A = Ab[cur];
  for (int e = t; e < k * k; e += blockDim.x) evec[e] = Vv[e];
  for (int j = t; j < k; j += blockDim.x) evals[j] = A[j * k + j];
}

// Select the p largest eigenvalues: theta[j], and the selection/rotation matrix
// sel (k x p, row-major) whose column j is the eigenvector of the j-th largest.  Lane i finds
// the rank of eigenvalue i (descending; ties by index, as a stable sort orders them).
__global__ void k_lmp_finish(const double* evals, const double* evec, int k, int p, double* theta, double* sel) {
  __shared__ int order[kMaxSketch];
  __shared__ double ev[kMaxSketch];
  const int t = threadIdx.x;
  if (t < k) ev[t] = evals[t];
  __syncthreads();
  if (t < k) {
    int rank = 0;
    for (int i = 0; i < k; ++i) rank += (ev[i] > ev[t]) || (ev[i] == ev[t] && i < t);
    order[rank] = t;
  }
  __syncthreads();
  if (t < p) theta[t] = ev[order[t]];
  for (int e = t; e < k * p; e += blockDim.x) {
    const int a = e / p, j = e % p;
    sel[a * p + j] = evec[a * k + order[j]];
  }
}

// G = X^T Y (row-major k x k, k = k1 + k2 <= 16) over m rows on an NT-thread workgroup by FP64
// MFMA, where X = [A1 A2] and Y = [B1 B2] are the column blocks of k1 and k2 columns: each
// wavefront takes blocks of 4 rows (wave w of NW: rows 4 w, 4 w + 4 NW, ...) into one
// v_mfma_f64_16x16x4f64 each (lane l brings column l % 16 of row 4 b + l / 16 of X and of Y: the
// A operand (row l % 16, k l / 16) is X^T, the B operand (k l / 16, col l % 16) is Y), U blocks'
// loads in flight before their products; then the NW wavefront tiles are added in a fixed order
// (wave w + NW / 2's into wave w's, then the NW / 2 sums in order).
// part: NW / 2 x 256 doubles of LDS; G complete on return.
typedef double small_d4 __attribute__((ext_vector_type(4)));
template <int NT>
__device__ inline void gram_mfma2(Strided A1, Strided A2, Strided B1, Strided B2, int64_t m, int k1, int k2,
                                  double* part, double* G) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = lane & 15, kk = lane >> 4;
  const int k = k1 + k2;
  const bool first = c < k1;
  const Strided A = first ? A1 : A2, B = first ? B1 : B2;
  const int cc = first ? c : c - k1;
  // this lane's column of X and of Y (rows at stride rs; m, rs and the column offsets fit 32 bits)
  const double* ac = A.ptr + (c < k ? cc * A.cs : 0);
  const double* bc = B.ptr + (c < k ? cc * B.cs : 0);
  const int ars = (int)A.rs, brs = (int)B.rs, mm = (int)m;
  // four independent accumulation chains, added at the end
  small_d4 acc[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = small_d4{0.0, 0.0, 0.0, 0.0};
  constexpr int U = NT >= 1024 ? 8 : 16;  // within 128 registers on 1024 threads
  for (int r0 = 4 * wave + kk; r0 - kk < mm; r0 += 4 * NW * U) {
    double a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 4 * NW * u;
      const bool ok = c < k && r < mm;
      a[u] = ok ? ac[r * ars] : 0.0;
      b[u] = ok ? bc[r * brs] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u % 4] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc[u % 4], 0, 0, 0);
  }
  // D register v: (row 4 v + lane / 16, col lane % 16)
  static_assert(NW >= 2 && NW % 2 == 0, "tiles added in pairs");
  constexpr int NH = NW / 2;
  double tv[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) tv[v] = (acc[0][v] + acc[1][v]) + (acc[2][v] + acc[3][v]);
  if (wave >= NH) {
#pragma unroll
    for (int v = 0; v < 4; ++v) part[(wave - NH) * 256 + (4 * v + kk) * 16 + c] = tv[v];
  }
  __syncthreads();
  if (wave < NH) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double* pp = part + wave * 256 + (4 * v + kk) * 16 + c;
      *pp = tv[v] + *pp;
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += NT) {
    const int i = (e / k) * 16 + e % k;
    double t = part[i];
#pragma unroll
    for (int w = 1; w < NH; ++w) t += part[w * 256 + i];
    G[e] = t;
  }
  __syncthreads();
}

template <int NT>
__device__ inline void gram_mfma(Strided A, Strided B, int64_t m, int k, double* part, double* G) {
  gram_mfma2<NT>(A, A, B, B, m, k, 0, part, G);
}

// The whole Gram matrix in one launch for k <= 16 (instead of partials + reduction).
__global__ __launch_bounds__(256) void k_gram_small(Strided A, Strided B, int64_t m, int k, double* __restrict__ G) {
  __shared__ double part[2 * 256];
  gram_mfma<256>(A, B, m, k, part, G);
}

// ----------------------------------------------------------- small bases on one workgroup
// With at most 8 sketch columns (p + oversample) the setup's small dense steps run as two
// launches: Cholesky-QR twice of Y = S Omega, then the Rayleigh quotient T = Qb^T (S Qb), its
// eigendecomposition, the top-p selection, the Ritz vectors Phi, S Phi and their three Gram
// blocks; the same arithmetic as the step-per-launch chain.

// Lane l's value of a double, to every lane (l uniform).
__device__ inline double small_readlane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Lane src's value of a double, for each lane (ds_bpermute on both halves).
__device__ inline double lane_shfl(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Upper Cholesky factor of the symmetric PSD k x k matrix G (row-major) on the first wavefront,
// lane i K + j holding entry (i, j): R[a*k+b] for b >= a (zero below) and 1 / R[a*k+a] in rinv[a]
// (zero for a dependent column).  A dependent column (pivot <= kCholDrop max diag G) gets a zero
// row; false when a pivot is not finite (the same in every lane).  Step c: the pivot by readlane,
// row c scaled, then the trailing block updated with row c's entries by two lane exchanges.
template <int K>
__device__ inline bool chol_upper_wave(const double* G, int k, double* R, double* rinv) {
  static_assert(K * K <= 64, "one entry a lane");
  const int lane = threadIdx.x & 63, i = lane / K, j = lane % K;
  const bool in = lane < K * K && i < k && j < k;
  double a = in ? G[i * k + j] : 0.0;
  double gmax = 0.0;
#pragma unroll
  for (int d = 0; d < K; ++d)
    if (d < k) gmax = fmax(gmax, small_readlane(a, d * K + d));
  bool ok = true;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    if (c < k) {
      const double d = small_readlane(a, c * K + c);
      if (!isfinite(d)) ok = false;
      const double rcc = (d > kCholDrop * gmax) ? sqrt(d) : 0.0;
      const double inv = rcc > 0.0 ? 1.0 / rcc : 0.0;
      if (i == c) a = j == c ? rcc : (j > c ? a * inv : a);
      const double rci = lane_shfl(a, c * K + i), rcj = lane_shfl(a, c * K + j);
      if (in && i > c && j >= i) a -= rci * rcj;
      if (lane == 0) rinv[c] = inv;
    }
  }
  if (in) R[i * k + j] = j >= i ? a : 0.0;
  return ok;
}

// Leading dimension of a staged m-row block in LDS: m rounded up to 32 plus 4 doubles, so that the
// 16 columns x 4 rows a wavefront reads for an FP64 MFMA fall in distinct banks.
__host__ __device__ constexpr int small_lp(int64_t m) { return (int)(((m + 31) / 32) * 32 + 4); }

// Columns [0, k) of the column-major m-row matrices A and B (leading dimension ld; B may be
// null) into dA and dB (leading dimension lp): a thread loads every column of its rows at once
// (2 K loads in flight) and stores them.
template <int NT, int K>
__device__ inline void stage_cols(const double* __restrict__ A, const double* __restrict__ B, int64_t ld, int64_t m,
                                  int k, double* dA, double* dB, int lp) {
  const int mm = (int)m, l = (int)ld;
  for (int r = threadIdx.x; r < mm; r += NT) {
    double va[K], vb[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      va[c] = c < k ? A[c * l + r] : 0.0;
      vb[c] = (B && c < k) ? B[c * l + r] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < K; ++c) {
      if (c < k) {
        dA[c * lp + r] = va[c];
        if (B) dB[c * lp + r] = vb[c];
      }
    }
  }
}

// Q = orth(Y) by Cholesky-QR twice: G = X^T X, X <- X R^{-1} (each row q solves q R = x by
// forward substitution), first with X = Y, then with X = Q.  Y and Q column-major, leading
// dimension ld.  With stage set the working copy lives in dynamic LDS (m x k, leading
// dimension m): one read of Y and one write of Q; otherwise Q itself is the working copy (a
// thread writes and later reads the same rows, tid + 1024 i; the Gram passes read every row after
// the barrier that ends the previous pass).
constexpr int kSmallNT = 1024;

template <int K>
__global__ __launch_bounds__(kSmallNT) void k_cholqr2_small(const double* __restrict__ Y, int64_t m, int k, int64_t ld,
                                                       double* __restrict__ Q, double* __restrict__ Q2, int32_t* flags,
                                                       int stage) {
  extern __shared__ __attribute__((aligned(16))) double xs[];
  __shared__ double part[kSmallNT / 128 * 256];
  __shared__ double G[K * K], R[K * K], Rinv[K];
  const int lp = small_lp(m);
  double* X = stage ? xs : Q;
  const int64_t lx = stage ? lp : ld;
  if (stage) {
    stage_cols<kSmallNT, K>(Y, nullptr, ld, m, k, xs, nullptr, lp);
    __syncthreads();
  }
  for (int pass = 0; pass < 2; ++pass) {
    const double* src = (pass == 0 && !stage) ? Y : X;
    const int64_t ls = (pass == 0 && !stage) ? ld : lx;
    gram_mfma<kSmallNT>(Strided{src, 1, ls}, Strided{src, 1, ls}, m, k, part, G);
    if (threadIdx.x < 64) {
      const bool ok = chol_upper_wave<K>(G, k, R, Rinv);
      if (threadIdx.x == 0 && !ok) atomicOr(flags, kFlagNumeric);
    }
    __syncthreads();
    const int ils = (int)ls, ilx = (int)lx;
    for (int r = threadIdx.x; r < (int)m; r += kSmallNT) {
      double x[K], q[K];
#pragma unroll
      for (int a = 0; a < K; ++a) x[a] = a < k ? src[a * ils + r] : 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        q[j] = 0.0;
        if (j < k) {
          double t = x[j];
#pragma unroll
          for (int a = 0; a < j; ++a) t -= q[a] * R[a * k + j];
          q[j] = t * Rinv[j];
        }
      }
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (j < k) X[j * ilx + r] = q[j];
    }
    __syncthreads();  // R is rewritten by the next pass
  }
  if (stage) {
    for (int r = threadIdx.x; r < (int)m; r += kSmallNT) {
      double v[K];
#pragma unroll
      for (int c = 0; c < K; ++c) v[c] = c < k ? xs[c * lp + r] : 0.0;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        if (c < k) {
          Q[c * (int)ld + r] = v[c];
          if (Q2) Q2[c * (int)ld + r] = v[c];
        }
      }
    }
  } else if (Q2) {  // a thread copies the rows it wrote
    for (int c = 0; c < k; ++c)
      for (int r = threadIdx.x; r < (int)m; r += kSmallNT) Q2[c * (int)ld + r] = Q[c * (int)ld + r];
  }
}

// Partner of index i in step `step` of the round-robin ordering over ke (even) players: slot 0
// holds player 0, slot t > 0 player 1 + (t - 1 + step) mod (ke - 1), and slots t and ke - 1 - t
// are paired.  Indices >= ke partner themselves.
__device__ inline int jacobi_partner(int i, int step, int ke) {
  if (i >= ke) return i;
  const int slot = i == 0 ? 0 : 1 + ((i - 1 - step) % (ke - 1) + (ke - 1)) % (ke - 1);
  const int ps = ke - 1 - slot;
  return ps == 0 ? 0 : 1 + (ps - 1 + step) % (ke - 1);
}

// T = Qb^T (S Qb), its Jacobi eigendecomposition on the first wavefront (lane i K + j holds A_ij
// and V_ij; each step rotates the k/2 pairs of the round-robin ordering at once, in one exchange
// of entries between lanes: each lane forms the rotations of its row's and its column's pair),
// the p largest eigenpairs (ties by index), Phi = Qb V_p and
// S Phi = (S Qb) V_p in FP64, theta, and the Gram blocks Phi^T Phi, Phi^T S Phi, (S Phi)^T S Phi
// of those vectors into G.
template <int K, int PB>
__global__ __launch_bounds__(kSmallNT) void k_ritz_small(const double* __restrict__ Qb, const double* __restrict__ SQ,
                                                    int64_t m, int k, int p, int64_t ld, double* __restrict__ theta,
                                                    double* __restrict__ Phi, double* __restrict__ SPhi,
                                                    double* __restrict__ G, int stage) {
  static_assert(K * K <= 64 && PB <= K, "one matrix entry a lane");
  // with stage set, Qb and S Qb are read once into dynamic LDS (m x k each, leading dimension
  // small_lp(m)); Phi and S Phi then replace their first p columns there for the last Gram pass
  extern __shared__ __attribute__((aligned(16))) double xs[];
  __shared__ double part[kSmallNT / 128 * 256];
  __shared__ double T[K * K], V[K * K], ev[K], sel[K * PB], W[4 * PB * PB];
  __shared__ int order[K];
  const int tid = threadIdx.x;
  const int lp = small_lp(m);
  const double* Qs = stage ? xs : Qb;
  const double* SQs = stage ? xs + (int64_t)lp * k : SQ;
  const int64_t lq = stage ? lp : ld;
  if (stage) {
    stage_cols<kSmallNT, K>(Qb, SQ, ld, m, k, xs, xs + (int64_t)lp * k, lp);
    __syncthreads();
  }
  gram_mfma<kSmallNT>(Strided{Qs, 1, lq}, Strided{SQs, 1, lq}, m, k, part, T);
  if (tid < 64) {
    const int i = tid / K, j = tid % K;
    const bool in = tid < K * K && i < k && j < k;
    double a = in ? 0.5 * (T[i * k + j] + T[j * k + i]) : 0.0;
    double v = (in && i == j) ? 1.0 : 0.0;
    const int ke = k + (k & 1);
    // this lane's row and column partners at every step of a sweep (ke - 1 <= K - 1 steps)
    int prow[K], pcol[K];
#pragma unroll
    for (int st = 0; st < K; ++st) {
      prow[st] = st < ke - 1 ? jacobi_partner(i, st, ke) : i;
      pcol[st] = st < ke - 1 ? jacobi_partner(j, st, ke) : j;
    }
    for (int sweep = 0; sweep < 40; ++sweep) {
      const double off = wave_sum_dpp(in && i != j ? a * a : 0.0);
      const double dia = wave_sum_dpp(in && i == j ? a * a : 0.0);
      // relative off-diagonal norm 1e-14 (FP64 Ritz vectors)
      if (lane_shfl(off, 63) <= 1e-28 * lane_shfl(dia, 63)) break;
#pragma unroll
      for (int step = 0; step < K - 1; ++step) {
        if (step >= ke - 1) break;
        const int pi = prow[step], pj = pcol[step];
        const int p1 = min(i, pi), q1 = max(i, pi), p2 = min(j, pj), q2 = max(j, pj);
        // one exchange: the pivots of the row pair and of the column pair, the 2 x 2 block of A at
        // rows {i, pi} and columns {j, pj}, and V's column partner
        const double rpp = lane_shfl(a, p1 * K + p1), rqq = lane_shfl(a, q1 * K + q1);
        const double rpq = lane_shfl(a, p1 * K + q1);
        const double cpp = lane_shfl(a, p2 * K + p2), cqq = lane_shfl(a, q2 * K + q2);
        const double cpq = lane_shfl(a, p2 * K + q2);
        const double arj = lane_shfl(a, pi * K + j), aic = lane_shfl(a, i * K + pj);
        const double arc = lane_shfl(a, pi * K + pj), vc = lane_shfl(v, i * K + pj);
        double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0;
        if (q1 < k && q1 != p1 && rpq != 0.0) jacobi_cs(rpp, rqq, rpq, &c1, &s1);
        if (q2 < k && q2 != p2 && cpq != 0.0) jacobi_cs(cpp, cqq, cpq, &c2, &s2);
        // rows [p; q] <- [c -s; s c] [p; q] (entries j and pj of row i), then columns likewise;
        // V <- V J
        const double b = i <= pi ? c1 * a - s1 * arj : s1 * arj + c1 * a;
        const double bc = i <= pi ? c1 * aic - s1 * arc : s1 * arc + c1 * aic;
        a = j <= pj ? c2 * b - s2 * bc : s2 * bc + c2 * b;
        v = j <= pj ? c2 * v - s2 * vc : s2 * vc + c2 * v;
      }
    }
    if (in) V[i * K + j] = v;
    if (in && i == j) ev[i] = a;
  }
  __syncthreads();
  if (tid < k) {
    int rank = 0;
    for (int i = 0; i < k; ++i) rank += (ev[i] > ev[tid]) || (ev[i] == ev[tid] && i < tid);
    order[rank] = tid;
  }
  __syncthreads();
  if (tid < p) theta[tid] = ev[order[tid]];
  for (int e = tid; e < k * p; e += kSmallNT) sel[(e / p) * PB + e % p] = V[(e / p) * K + order[e % p]];
  __syncthreads();
  const int ilq = (int)lq, ild = (int)ld;
  for (int r = tid; r < (int)m; r += kSmallNT) {
    double q[K], sq[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
      q[a] = a < k ? Qs[a * ilq + r] : 0.0;
      sq[a] = a < k ? SQs[a * ilq + r] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < PB; ++jj) {
      if (jj < p) {
        double f = 0.0, g = 0.0;
#pragma unroll
        for (int a = 0; a < K; ++a) {
          if (a < k) {
            f += q[a] * sel[a * PB + jj];
            g += sq[a] * sel[a * PB + jj];
          }
        }
        Phi[jj * ild + r] = f;
        SPhi[jj * ild + r] = g;
        if (stage) {  // this thread read its rows of Qb and S Qb above
          xs[jj * ilq + r] = f;
          xs[(int64_t)lp * k + jj * ilq + r] = g;
        }
      }
    }
  }
  __syncthreads();  // every row of Phi and S Phi is written
  // the Gram of [Phi S Phi] (2p x 2p) in one pass; its blocks Phi^T Phi, Phi^T S Phi and
  // (S Phi)^T S Phi go to G
  const Strided Ph = stage ? Strided{xs, 1, lq} : Strided{Phi, 1, ld};
  const Strided SPh = stage ? Strided{xs + (int64_t)lp * k, 1, lq} : Strided{SPhi, 1, ld};
  gram_mfma2<kSmallNT>(Ph, SPh, Ph, SPh, m, p, p, part, W);
  const int p2 = 2 * p;
  for (int e = tid; e < 3 * p * p; e += kSmallNT) {
    const int blk = e / (p * p), a = (e % (p * p)) / p, b = e % p;
    const int row = blk == 2 ? p + a : a, col = blk == 0 ? b : p + b;
    G[e] = W[row * p2 + col];
  }
}

__global__ void k_min_reduce(const double* v, int64_t count, double* out) {
  __shared__ double red[256];
  double m = 1.0 / 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) m = fmin(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

hipError_t launch_sketch(uint64_t seed, int64_t m, int k, double* out, int64_t ld, hipStream_t st) {
  const int64_t cnt = m * k;
  hipLaunchKernelGGL(k_sketch, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, seed, m, k, out, ld);
  return hipGetLastError();
}

hipError_t launch_sketch_setup(uint64_t seed, int64_t m, int k, double* out, int64_t ld, int32_t* act, int32_t* nact,
                               double* sig, int nsig, hipStream_t st) {
  if (!out || !act || !nact || !sig || k < 1 || m < 1 || ld < m || nsig < k) return hipErrorInvalidValue;
  const int64_t cnt = std::max<int64_t>(ld * k, nsig);
  hipLaunchKernelGGL(k_sketch_setup, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, seed, m, k, out, ld, act,
                     nact, sig, nsig);
  return hipGetLastError();
}

int gram_chunks(int64_t m) { return (int)((m + kGramChunk - 1) / kGramChunk); }

hipError_t launch_gram(Strided A, Strided B, int64_t m, int k, double* G, double* scratch, hipStream_t st) {
  if (k < 1 || k > kMaxSketch || m < 1) return hipErrorInvalidValue;
  if (k <= 16 && m <= 8192) {
    hipLaunchKernelGGL(k_gram_small, dim3(1), dim3(256), 0, st, A, B, m, k, G);
    return hipGetLastError();
  }
  const int nchunks = gram_chunks(m);
  hipLaunchKernelGGL(k_gram_partial, dim3(nchunks), dim3(256), 0, st, A, B, m, k, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3((k * k + 255) / 256), dim3(256), 0, st, scratch, nchunks, k, G);
  return hipGetLastError();
}

hipError_t launch_chol_inv(double* G, int k, int32_t* flags, hipStream_t st) {
  if (k < 1 || k > kMaxSketch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(64), 0, st, G, k, flags);
  return hipGetLastError();
}

hipError_t launch_right_mult(Strided A, int64_t m, int k, const double* M, int kout, double* out, int64_t ors,
                             int64_t ocs, hipStream_t st) {
  const int64_t cnt = m * kout;
  hipLaunchKernelGGL(k_right_mult, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, A, m, k, M, kout, out, ors,
                     ocs);
  return hipGetLastError();
}

hipError_t launch_sym_eig(double* T, int k, double* evec, double* evals, hipStream_t st) {
  if (k < 1 || k > kMaxSketch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sym_eig, dim3(1), dim3(256), 0, st, T, k, evec, evals);
  return hipGetLastError();
}

hipError_t launch_lmp_finish(const double* evals, const double* evec, int k, int p, double* theta, double* sel,
                             hipStream_t st) {
  if (k < 1 || k > kMaxSketch || p > k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lmp_finish, dim3(1), dim3(64), 0, st, evals, evec, k, p, theta, sel);
  return hipGetLastError();
}

bool small_basis_fits(int k, int p, int64_t m) { return k >= 1 && k <= 8 && p >= 1 && p <= k && m >= 1 && m <= 8192; }
// the kernels index columns with 32-bit offsets
constexpr int64_t kSmallMaxLd = int64_t(1) << 26;

// dynamic LDS the small-basis kernels may take for a staged copy
constexpr size_t kSmallStage = 96 * 1024;
constexpr size_t kSmallStageRitz = 136 * 1024;

hipError_t launch_cholqr2_small(const double* Y, int64_t m, int k, int64_t ld, double* Q, double* Q2, int32_t* flags,
                                hipStream_t st) {
  if (!Y || !Q || !flags || ld < m || ld > kSmallMaxLd || !small_basis_fits(k, 1, m)) return hipErrorInvalidValue;
  const size_t bytes = (size_t)small_lp(m) * k * sizeof(double);
  const int stage = bytes <= kSmallStage ? 1 : 0;
  const size_t dyn = stage ? bytes : 0;
  const void* fn = k <= 4 ? (const void*)k_cholqr2_small<4> : (const void*)k_cholqr2_small<8>;
  static std::atomic<bool> raised[2] = {false, false};
  if (dyn > 64 * 1024 && !raised[k <= 4 ? 0 : 1].load()) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallStage);
    if (e != hipSuccess) return e;
    raised[k <= 4 ? 0 : 1].store(true);
  }
  if (k <= 4)
    hipLaunchKernelGGL(k_cholqr2_small<4>, dim3(1), dim3(kSmallNT), dyn, st, Y, m, k, ld, Q, Q2, flags, stage);
  else
    hipLaunchKernelGGL(k_cholqr2_small<8>, dim3(1), dim3(kSmallNT), dyn, st, Y, m, k, ld, Q, Q2, flags, stage);
  return hipGetLastError();
}

hipError_t launch_ritz_small(const double* Qb, const double* SQ, int64_t m, int k, int p, int64_t ld, double* theta,
                             double* Phi, double* SPhi, double* G, hipStream_t st) {
  if (!Qb || !SQ || !theta || !Phi || !SPhi || !G || ld < m || ld > kSmallMaxLd ||
      !small_basis_fits(k, p, m))
    return hipErrorInvalidValue;
  const size_t bytes = 2 * (size_t)small_lp(m) * k * sizeof(double);
  const int stage = bytes <= kSmallStageRitz ? 1 : 0;
  const size_t dyn = stage ? bytes : 0;
  const int which = k <= 4 ? 0 : (p <= 4 ? 1 : 2);
  const void* fn = which == 0 ? (const void*)k_ritz_small<4, 4>
                              : (which == 1 ? (const void*)k_ritz_small<8, 4> : (const void*)k_ritz_small<8, 8>);
  static std::atomic<bool> raised[3] = {false, false, false};
  if (dyn > 64 * 1024 && !raised[which].load()) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallStageRitz);
    if (e != hipSuccess) return e;
    raised[which].store(true);
  }
  if (which == 0)
    hipLaunchKernelGGL((k_ritz_small<4, 4>), dim3(1), dim3(kSmallNT), dyn, st, Qb, SQ, m, k, p, ld, theta, Phi, SPhi,
                       G, stage);
  else if (which == 1)
    hipLaunchKernelGGL((k_ritz_small<8, 4>), dim3(1), dim3(kSmallNT), dyn, st, Qb, SQ, m, k, p, ld, theta, Phi, SPhi,
                       G, stage);
  else
    hipLaunchKernelGGL((k_ritz_small<8, 8>), dim3(1), dim3(kSmallNT), dyn, st, Qb, SQ, m, k, p, ld, theta, Phi, SPhi,
                       G, stage);
  return hipGetLastError();
}

hipError_t launch_min_reduce(const double* v, int64_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(256), 0, st, v, count, out);
  return hipGetLastError();
}

}  // namespace infoesrf
