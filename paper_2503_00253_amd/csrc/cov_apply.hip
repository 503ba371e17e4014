// Localized covariance apply in operator form (Sec. 2.3, eq. 2.12) on gfx950 MFMA.
//
//   T[:, b] = P V[:, b] = sum_i z_i o L (z_i o V[:, b]),    P = L o (Z Z^T)
//
// L is a stationary stencil on an nz x nx grid.  For one output row tile of
// TM consecutive x positions in layer z, and one stencil layer offset dz,
// the rows of L restricted to the tile form a TM x (TM + 2bx) Toeplitz block
// whose entries come straight from the stencil table.  The apply is therefore
// a banded dense contraction
//
//   T[r, b] += sum_{i, k} (z_i[r] L[r, k]) (z_i[k] V[k, b])
//
// with the contraction index running jointly over members i and the K-window
// k.  Both operands are formed in registers from Z, V and the table: the
// member block z_i o V (n x N*B) never exists in memory.  The output row
// scaling z_i[r] is folded into the A operand so the MFMA accumulates P V
// directly, without a per-member epilogue.
//
// Work decomposition: one wavefront owns RB row blocks of 16 rows (TM = 16 RB
// consecutive x in one layer) and 16 systems; the block's four waves own four
// consecutive row tiles.  Row blocks skip K steps that lie outside their band,
// so the padded MFMA work per row block is (16 + 2bx + 3) / (2bx + 1) of the
// band's.
#include "internal.hpp"

namespace infoesrf {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// zero padding on each side of a table row: a fragment that overlaps the band reads
// offsets d = k - r in [base - 15, base + 3] with base in [-3, 2bx + 15], so up to 18
// entries beyond either end of the band.
constexpr int kPad = 20;

template <typename T>
struct Mfma;

// v_mfma_f64_16x16x4f64: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
// D register v of lane l -> (row 4v + l/16, col l%16).
template <>
struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ inline acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int lane, int v) { return 4 * v + (lane >> 4); }
};

// v_mfma_f32_16x16x4f32: A, B as above; D register v of lane l -> (row 4(l/16) + v, col l%16).
template <>
struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ inline acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T>
__device__ inline const T* table_ptr(const Grid& g);
template <>
__device__ inline const double* table_ptr<double>(const Grid& g) { return g.table; }
template <>
__device__ inline const float* table_ptr<float>(const Grid& g) { return g.table32; }

__device__ inline int wrap_mod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

template <typename T, int RB>
__global__ __launch_bounds__(256) void k_cov_stencil(Grid g, const T* __restrict__ Z, int64_t ldz, int N,
                                                     const T* __restrict__ V, int64_t ldv, int B,
                                                     const int32_t* __restrict__ Bdev, T* __restrict__ Tout,
                                                     int64_t ldt, int tiles_per_layer, int ntiles,
                                                     ProfDev prof) {
  if (Bdev) B = *Bdev;  // active-system count produced on the device
  if (prof.vectors && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    atomicAdd(prof.vectors, (unsigned long long)B);
    atomicAdd(prof.flops, (double)B * prof.flops_per_vector);
  }
  if ((int)blockIdx.y * 16 >= B) return;
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int TM = 16 * RB;
  extern __shared__ unsigned char smem_raw[];
  T* tab = reinterpret_cast<T*>(smem_raw);

  const int bx = g.bx, bz = g.bz;
  const int tw = 2 * bx + 1 + 2 * kPad;  // padded table row width
  const T* gtab = table_ptr<T>(g);
  for (int t = threadIdx.x; t < (2 * bz + 1) * tw; t += blockDim.x) {
    const int row = t / tw, c = t % tw - kPad;
    tab[t] = (c >= 0 && c <= 2 * bx) ? gtab[row * (2 * bx + 1) + c] : T(0);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= ntiles) return;
  const int z = tile / tiles_per_layer;
  const int x0 = (tile % tiles_per_layer) * TM;
  const int nx = g.nx, nz = g.nz;
  const int b = blockIdx.y * 16 + (lane & 15);  // this lane's B column (< padded B)
  const int lrow = lane & 15;                   // A operand row within a row block
  const int lk = lane >> 4;                     // operand k within a K step

  acc_t acc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = acc_t{0, 0, 0, 0};

  const int KW = TM + 2 * bx;
  const int nK = (KW + 3) / 4;

  for (int dz = -bz; dz <= bz; ++dz) {
    int zz = z + dz;
    if (g.pz) {
      zz = wrap_mod(zz, nz);
    } else if (zz < 0 || zz >= nz) {
      continue;
    }
    const T* trow = tab + (dz + bz) * tw + kPad;
    const int64_t lay = (int64_t)zz * nx;
    for (int i = 0; i < N; ++i) {
      const T* zc = Z + (int64_t)i * ldz;
      T zr[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int xr = x0 + 16 * rb + lrow;
        zr[rb] = (xr < nx) ? zc[(int64_t)z * nx + xr] : T(0);
      }
      // one-step software prefetch of the B operand
      auto load_b = [&](int kk) -> T {
        const int kl = 4 * kk + lk;
        int kx = x0 - bx + kl;
        if (g.px) {
          kx = wrap_mod(kx, nx);
        } else if (kx < 0 || kx >= nx) {
          return T(0);
        }
        if (kl >= KW) return T(0);
        const int64_t kidx = lay + kx;
        return zc[kidx] * V[kidx * ldv + b];
      };
      T bnext = load_b(0);
      for (int kk = 0; kk < nK; ++kk) {
        const T bval = bnext;
        if (kk + 1 < nK) bnext = load_b(kk + 1);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int base = 4 * kk - 16 * rb;
          if (base + 3 >= 0 && base - 15 <= 2 * bx) {
            const T a = zr[rb] * trow[base + lk - lrow];
            acc[rb] = Mfma<T>::step(a, bval, acc[rb]);
          }
        }
      }
    }
  }

  if (b >= B) return;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int x = x0 + 16 * rb + Mfma<T>::out_row(lane, v);
      if (x < nx) Tout[((int64_t)z * nx + x) * ldt + b] = acc[rb][v];
    }
  }
}

template <typename T, int RB>
hipError_t launch_typed(const Grid& g, const T* Z, int64_t ldz, int64_t N, const T* V, int64_t ldv, int64_t B,
                        const int32_t* Bdev, T* Tout, int64_t ldt, hipStream_t st, const ProfDev& prof) {
  constexpr int TM = 16 * RB;
  const int tiles_per_layer = (g.nx + TM - 1) / TM;
  const int ntiles = tiles_per_layer * g.nz;
  const size_t smem = sizeof(T) * (size_t)(2 * g.bz + 1) * (2 * g.bx + 1 + 2 * kPad);
  dim3 grid((ntiles + 3) / 4, (unsigned)((B + 15) / 16));
  hipLaunchKernelGGL((k_cov_stencil<T, RB>), grid, dim3(256), smem, st, g, Z, ldz, (int)N, V, ldv, (int)B, Bdev,
                     Tout, ldt, tiles_per_layer, ntiles, prof);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb(int rows_per_wave, const Grid& g, const T* Z, int64_t ldz, int64_t N, const T* V, int64_t ldv,
                     int64_t B, const int32_t* Bdev, T* Tout, int64_t ldt, hipStream_t st, const ProfDev& pf) {
  switch (rows_per_wave) {
    case 16: return launch_typed<T, 1>(g, Z, ldz, N, V, ldv, B, Bdev, Tout, ldt, st, pf);
    case 32: return launch_typed<T, 2>(g, Z, ldz, N, V, ldv, B, Bdev, Tout, ldt, st, pf);
    case 64: return launch_typed<T, 4>(g, Z, ldz, N, V, ldv, B, Bdev, Tout, ldt, st, pf);
    case 128: return launch_typed<T, 8>(g, Z, ldz, N, V, ldv, B, Bdev, Tout, ldt, st, pf);
    default: return hipErrorInvalidValue;
  }
}

// Dense L (small n, tests): T[r, b] = sum_i z_i[r] sum_k L[r,k] z_i[k] V[k,b]; one thread per (r, b).
__global__ void k_cov_dense(const double* __restrict__ L, const double* __restrict__ Z, int64_t n, int64_t N,
                            const double* __restrict__ V, int64_t ldv, int64_t B, double* __restrict__ T,
                            int64_t ldt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * B) return;
  const int64_t r = t / B, b = t % B;
  double acc = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    double inner = 0.0;
    for (int64_t k = 0; k < n; ++k) inner += L[r + k * n] * Z[k + i * n] * V[k * ldv + b];
    acc += Z[r + i * n] * inner;
  }
  T[r * ldt + b] = acc;
}

}  // namespace

hipError_t launch_cov_stencil(Prec prec, const Grid& g, const void* Z, int64_t ldz, int64_t N, const void* V,
                              int64_t ldv, int64_t B, const int32_t* Bdev, void* T, int64_t ldt, int rows_per_wave,
                              hipStream_t st, const ProfDev* prof) {
  if (B <= 0) return hipSuccess;
  const ProfDev pf = prof ? *prof : ProfDev{nullptr, nullptr, 0.0};
  switch (prec) {
    case Prec::F64:
      return launch_rb<double>(rows_per_wave, g, (const double*)Z, ldz, N, (const double*)V, ldv, B, Bdev,
                               (double*)T, ldt, st, pf);
    case Prec::F32:
      return launch_rb<float>(rows_per_wave, g, (const float*)Z, ldz, N, (const float*)V, ldv, B, Bdev, (float*)T,
                              ldt, st, pf);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cov_dense(const double* L, const double* Z, int64_t n, int64_t N, const double* V, int64_t ldv,
                            int64_t B, double* T, int64_t ldt, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const int64_t cnt = n * B;
  hipLaunchKernelGGL(k_cov_dense, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, L, Z, n, N, V, ldv, B, T,
                     ldt);
  return hipGetLastError();
}

}  // namespace infoesrf
