// Limited-memory preconditioner setup (Appendix E): Ritz pairs of S from a
// randomized symmetric eigendecomposition (Halko, Martinsson & Tropp: range
// finder followed by the direct eigendecomposition of the projected matrix).
//
//   Y = S Omega, Qb = orth(Y) (Cholesky-QR applied twice), T = Qb^T (S Qb),
//   T = V diag(lambda) V^T, Phi = Qb V_p, S Phi = (S Qb) V_p, theta = lambda_p.
//
// All small dense steps run on one workgroup so the setup needs no host round
// trip and can be captured in a HIP graph.
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

// partial Gram over a row chunk: scratch[chunk][a*k+b]
__global__ void k_gram_partial(Strided A, Strided B, int64_t m, int k, int chunk_rows, double* __restrict__ scratch) {
  const int64_t r0 = blockIdx.x * (int64_t)chunk_rows;
  const int64_t r1 = min<int64_t>(m, r0 + chunk_rows);
  for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
    const int a = t / k, b = t % k;
    double acc = 0.0;
    for (int64_t r = r0; r < r1; ++r) acc += A.ptr[r * A.rs + a * A.cs] * B.ptr[r * B.rs + b * B.cs];
    scratch[blockIdx.x * (int64_t)k * k + t] = acc;
  }
}

__global__ void k_gram_reduce(const double* __restrict__ scratch, int nchunks, int k, double* __restrict__ G) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * k) return;
  double acc = 0.0;
  for (int c = 0; c < nchunks; ++c) acc += scratch[(int64_t)c * k * k + t];
  G[t] = acc;
}

// G (k x k, row-major, SPD) -> inverse of its upper Cholesky factor R (G = R^T R), in place.
__global__ void k_chol_inv(double* G, int k, int32_t* flags) {
  __shared__ double R[kMaxSketch * kMaxSketch];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < k * k; e += blockDim.x) R[e] = G[e];
  __syncthreads();
  // right-looking Cholesky, column j
  for (int j = 0; j < k; ++j) {
    if (t == 0) {
      const double d = R[j * k + j];
      if (!(d > 0.0)) {
        bad = 1;
        R[j * k + j] = 1.0;
      } else {
        R[j * k + j] = sqrt(d);
      }
    }
    __syncthreads();
    const double rjj = R[j * k + j];
    for (int c = j + 1 + t; c < k; c += blockDim.x) R[j * k + c] /= rjj;
    __syncthreads();
    for (int e = t; e < (k - j - 1) * (k - j - 1); e += blockDim.x) {
      const int a = j + 1 + e / (k - j - 1), b = j + 1 + e % (k - j - 1);
      if (b >= a) R[a * k + b] -= R[j * k + a] * R[j * k + b];
    }
    __syncthreads();
  }
  // R is upper triangular in R[a*k+b], b >= a.  Invert by columns: Rinv[:, c] solves R x = e_c.
  for (int c = t; c < k; c += blockDim.x) {
    double x[kMaxSketch];
    for (int a = k - 1; a >= 0; --a) {
      double s = (a == c) ? 1.0 : 0.0;
      for (int b = a + 1; b < k; ++b) s -= R[a * k + b] * x[b];
      x[a] = (a <= c) ? s / R[a * k + a] : 0.0;
    }
    for (int a = 0; a < k; ++a) G[a * k + c] = x[a];
  }
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

// Jacobi eigendecomposition of a small symmetric matrix on one workgroup with the
// round-robin (tournament) ordering: each step rotates k/2 disjoint index pairs at
// once, k-1 steps make a sweep in which every pair is visited once.
// T (k x k row-major) is read; evec[a*k + j] = component a of eigenvector j.
__global__ void k_sym_eig(double* T, int k, double* evec, double* evals) {
  __shared__ double A[kMaxSketch * kMaxSketch];
  __shared__ double Vv[kMaxSketch * kMaxSketch];
  __shared__ double cs_c[kMaxSketch / 2], cs_s[kMaxSketch / 2];
  __shared__ int pp[kMaxSketch / 2], qq[kMaxSketch / 2];
  __shared__ double red_off[256], red_dia[256];
  const int t = threadIdx.x;
  const int ke = k + (k & 1);  // even number of players; index k (if odd) is a dummy
  const int half = ke / 2;
  for (int e = t; e < k * k; e += blockDim.x) {
    A[e] = 0.5 * (T[e] + T[(e % k) * k + e / k]);
    Vv[e] = (e / k == e % k) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int e = t; e < k * k; e += blockDim.x) {
      const double v = A[e] * A[e];
      if (e / k == e % k) dia += v;
      else off += v;
    }
    red_off[t] = off;
    red_dia[t] = dia;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (t < w) {
        red_off[t] += red_off[t + w];
        red_dia[t] += red_dia[t + w];
      }
      __syncthreads();
    }
    const bool conv = red_off[0] <= 1e-30 * red_dia[0];
    __syncthreads();
    if (conv) break;
    for (int step = 0; step < ke - 1; ++step) {
      if (t < half) {
        // players: slot 0 fixed, slots 1..ke-1 rotate by `step`
        auto player = [&](int slot) { return slot == 0 ? 0 : 1 + (slot - 1 + step) % (ke - 1); };
        int p = player(t), q = player(ke - 1 - t);
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        double c = 1.0, sn = 0.0;
        if (q < k) {
          const double apq = A[p * k + q];
          if (apq != 0.0) {
            const double tau = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
          }
        }
        pp[t] = p;
        qq[t] = (q < k) ? q : p;
        cs_c[t] = c;
        cs_s[t] = (q < k) ? sn : 0.0;
      }
      __syncthreads();
      // rows p, q of every pair
      for (int e = t; e < half * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        const double sn = cs_s[i];
        if (sn == 0.0) continue;
        const int p = pp[i], q = qq[i];
        const double c = cs_c[i];
        const double ap = A[p * k + j], aq = A[q * k + j];
        A[p * k + j] = c * ap - sn * aq;
        A[q * k + j] = sn * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of every pair, and the eigenvector columns
      for (int e = t; e < half * k; e += blockDim.x) {
        const int i = e / k, j = e % k;
        const double sn = cs_s[i];
        if (sn == 0.0) continue;
        const int p = pp[i], q = qq[i];
        const double c = cs_c[i];
        const double ap = A[j * k + p], aq = A[j * k + q];
        A[j * k + p] = c * ap - sn * aq;
        A[j * k + q] = sn * ap + c * aq;
        const double vp = Vv[j * k + p], vq = Vv[j * k + q];
        Vv[j * k + p] = c * vp - sn * vq;
        Vv[j * k + q] = sn * vp + c * vq;
      }
      __syncthreads();
    }
  }
  for (int e = t; e < k * k; e += blockDim.x) evec[e] = Vv[e];
  for (int j = t; j < k; j += blockDim.x) evals[j] = A[j * k + j];
}

// Select the p largest eigenvalues: theta[j], and the selection/rotation matrix
// sel (k x p, row-major) whose column j is the eigenvector of the j-th largest.
__global__ void k_lmp_finish(const double* evals, const double* evec, int k, int p, double* theta, double* sel) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int order[kMaxSketch];
  for (int j = 0; j < k; ++j) order[j] = j;
  for (int a = 1; a < k; ++a) {  // insertion sort, descending, stable
    const int v = order[a];
    int b = a - 1;
    while (b >= 0 && evals[order[b]] < evals[v]) {
      order[b + 1] = order[b];
      --b;
    }
    order[b + 1] = v;
  }
  for (int j = 0; j < p; ++j) {
    theta[j] = evals[order[j]];
    for (int a = 0; a < k; ++a) sel[a * p + j] = evec[a * k + order[j]];
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

hipError_t launch_gram(Strided A, Strided B, int64_t m, int k, double* G, double* scratch, hipStream_t st) {
  const int chunk = 128;
  const int nchunks = (int)((m + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_gram_partial, dim3(nchunks), dim3(256), 0, st, A, B, m, k, chunk, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3((k * k + 255) / 256), dim3(256), 0, st, scratch, nchunks, k, G);
  return hipGetLastError();
}

hipError_t launch_chol_inv(double* G, int k, int32_t* flags, hipStream_t st) {
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
  hipLaunchKernelGGL(k_sym_eig, dim3(1), dim3(256), 0, st, T, k, evec, evals);
  return hipGetLastError();
}

hipError_t launch_lmp_finish(const double* evals, const double* evec, int k, int p, double* theta, double* sel,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_lmp_finish, dim3(1), dim3(64), 0, st, evals, evec, k, p, theta, sel);
  return hipGetLastError();
}

hipError_t launch_min_reduce(const double* v, int64_t count, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(256), 0, st, v, count, out);
  return hipGetLastError();
}

}  // namespace infoesrf
