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
#include <atomic>
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

// LDS row padding of the staged V window (64 bytes) so the four K rows a
// wavefront reads in one step fall on different banks.
template <typename T>
constexpr int vpad() { return 64 / (int)sizeof(T); }

// Block tile: TM = 16 RB output rows of one layer, NS = 16 SB systems.  The
// four wavefronts of a block split the members (wave w takes members
// j = w, w+4, ...) and each accumulates the whole TM x NS tile; a final
// cross-wave reduction in LDS sums the four partial tiles.  V and Z are staged
// in LDS one K-chunk (KC rows of the K-window) and one member chunk (MC
// members) at a time, so the LDS footprint does not grow with the stencil.
template <typename T, int RB, int SB>
__global__ __launch_bounds__(256) void k_cov_stencil(Grid g, const T* __restrict__ Z, int64_t ldz, int N,
                                                     const T* __restrict__ V, int64_t ldv, int64_t vcols, int B,
                                                     const int32_t* __restrict__ Bdev, T* __restrict__ Tout,
                                                     int64_t ldt, int tiles_per_layer, int KC, int MC,
                                                     ProfDev prof, int32_t* __restrict__ zero_counter) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int TM = 16 * RB;
  constexpr int NS = 16 * SB;
  constexpr int VS = NS + vpad<T>();
  if (Bdev) B = *Bdev;  // active-system count produced on the device
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    if (zero_counter) {  // list and live counters of the next PCG step (nobody reads them now)
      zero_counter[0] = 0;
      zero_counter[1] = 0;
    }
    if (prof.vectors) {
      atomicAdd(prof.vectors, (unsigned long long)B);
      atomicAdd(prof.flops, (double)B * prof.flops_per_vector);
      atomicAdd(prof.bytes, (double)B * prof.bytes_per_vector);
    }
  }
  const int b0 = blockIdx.y * NS;
  if (b0 >= B) return;

  extern __shared__ unsigned char smem_raw[];
  const int bx = g.bx, bz = g.bz;
  const int tw = 2 * bx + 1 + 2 * kPad;
  T* tab = reinterpret_cast<T*>(smem_raw);
  T* Vw = tab + (2 * bz + 1) * tw;  // KC x VS
  T* Zw = Vw + KC * VS;             // MC x KC
  T* Zr = Zw + MC * KC;             // MC x TM
  int* kxs = reinterpret_cast<int*>(Zr + MC * TM);  // KC: wrapped x of each chunk row, -1 outside

  const T* gtab = table_ptr<T>(g);
  for (int t = threadIdx.x; t < (2 * bz + 1) * tw; t += blockDim.x) {
    const int row = t / tw, c = t % tw - kPad;
    tab[t] = (c >= 0 && c <= 2 * bx) ? gtab[row * (2 * bx + 1) + c] : T(0);
  }

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tile = blockIdx.x;
  const int z = tile / tiles_per_layer;
  const int x0 = (tile % tiles_per_layer) * TM;
  const int nx = g.nx, nz = g.nz;
  const int lrow = lane & 15;
  const int lk = lane >> 4;
  const int KW = TM + 2 * bx;

  acc_t acc[RB][SB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) acc[rb][sb] = acc_t{0, 0, 0, 0};

  for (int m0 = 0; m0 < N; m0 += MC) {
    const int mcn = min(MC, N - m0);
    __syncthreads();
    // output-row scales z_i[r] of this member chunk (layer z)
    for (int t = threadIdx.x; t < MC * TM; t += blockDim.x) {
      const int j = t / TM, r = t % TM;
      const int xr = x0 + r;
      Zr[t] = (j < mcn && xr < nx) ? Z[(int64_t)(m0 + j) * ldz + (int64_t)z * nx + xr] : T(0);
    }
    for (int dz = -bz; dz <= bz; ++dz) {
      int zz = z + dz;
      if (g.pz) {
        zz = wrap_mod(zz, nz);
      } else if (zz < 0 || zz >= nz) {
        continue;
      }
      const T* trow = tab + (dz + bz) * tw + kPad;
      const int64_t lay = (int64_t)zz * nx;
      for (int k0 = 0; k0 < KW; k0 += KC) {
        __syncthreads();
        for (int kl = threadIdx.x; kl < KC; kl += blockDim.x) {
          const int kw = k0 + kl;
          int kx = x0 - bx + kw;
          bool ok = kw < KW;
          if (g.px) kx = wrap_mod(kx, nx);
          else ok = ok && kx >= 0 && kx < nx;
          kxs[kl] = ok ? kx : -1;
        }
        __syncthreads();
        // stage V rows k0..k0+KC of the K-window (systems b0..b0+NS; V is system-major, so the
        // lanes of a wavefront read consecutive k of one column) and the matching Z rows
        const int lw = threadIdx.x & 63, wv = threadIdx.x >> 6;
        for (int c = wv; c < NS; c += 4) {
          const bool colok = b0 + c < vcols;  // columns past the buffer width are not read
          const T* vcol = V + (int64_t)(b0 + c) * ldv + lay;
          for (int kl = lw; kl < KC; kl += 64) {
            const int kx = kxs[kl];
            Vw[kl * VS + c] = (colok && kx >= 0) ? vcol[kx] : T(0);
          }
        }
        for (int j = wv; j < MC; j += 4) {
          const bool jok = j < mcn;
          const T* zcol = Z + (int64_t)(m0 + (jok ? j : 0)) * ldz + lay;
          for (int kl = lw; kl < KC; kl += 64) {
            const int kx = kxs[kl];
            Zw[j * KC + kl] = (jok && kx >= 0) ? zcol[kx] : T(0);
          }
        }
        __syncthreads();
        const int kk0 = k0 >> 2;
        const int nkk = KC >> 2;
        for (int j = wave; j < mcn; j += 4) {
          T zr[RB];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) zr[rb] = Zr[j * TM + 16 * rb + lrow];
          const T* zk_row = Zw + j * KC;
          for (int kl4 = 0; kl4 < nkk; ++kl4) {
            const int kl = 4 * kl4 + lk;
            const T zk = zk_row[kl];
            T bv[SB];
#pragma unroll
            for (int sb = 0; sb < SB; ++sb) bv[sb] = zk * Vw[kl * VS + 16 * sb + lrow];
            const int kk = kk0 + kl4;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              const int base = 4 * kk - 16 * rb;
              if (base + 3 >= 0 && base - 15 <= 2 * bx) {
                const T a = zr[rb] * trow[base + lk - lrow];
#pragma unroll
                for (int sb = 0; sb < SB; ++sb) acc[rb][sb] = Mfma<T>::step(a, bv[sb], acc[rb][sb]);
              }
            }
          }
        }
      }
    }
  }

  // cross-wave reduction of the four partial tiles
  __syncthreads();
  T* red = Vw;  // reuse: needs 4 * 64 * RB * SB * 4 values (checked by the launcher)
  constexpr int PER = RB * SB * 4;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[((wave * PER) + (rb * SB + sb) * 4 + v) * 64 + lane] = acc[rb][sb][v];
  __syncthreads();
  // each wave writes a quarter of the tile's fragments
  for (int f = wave; f < RB * SB; f += 4) {
    const int rb = f / SB, sb = f % SB;
    const int b = b0 + 16 * sb + (lane & 15);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T s = T(0);
#pragma unroll
      for (int w = 0; w < 4; ++w) s += red[((w * PER) + f * 4 + v) * 64 + lane];
      const int x = x0 + 16 * rb + Mfma<T>::out_row(lane, v);
      if (x < nx && b < B) Tout[(int64_t)b * ldt + (int64_t)z * nx + x] = s;
    }
  }
}

template <typename T, int RB, int SB>
size_t smem_bytes(const Grid& g, int KC, int MC) {
  constexpr int TM = 16 * RB, NS = 16 * SB, VS = NS + vpad<T>();
  const size_t stage = (size_t)KC * VS + (size_t)MC * KC + (size_t)MC * TM +
                       ((size_t)KC * sizeof(int) + sizeof(T) - 1) / sizeof(T);
  const size_t red = (size_t)4 * 64 * RB * SB * 4;
  return sizeof(T) * ((size_t)(2 * g.bz + 1) * (2 * g.bx + 1 + 2 * kPad) + (stage > red ? stage : red));
}

template <typename T, int RB, int SB>
hipError_t launch_typed(const Grid& g, const T* Z, int64_t ldz, int64_t N, const T* V, int64_t ldv, int64_t vcols,
                        int64_t B, const int32_t* Bdev, T* Tout, int64_t ldt, hipStream_t st, const ProfDev& prof,
                        int32_t* zero_counter) {
  constexpr int TM = 16 * RB, NS = 16 * SB;
  const int tiles_per_layer = (g.nx + TM - 1) / TM;
  const int ntiles = tiles_per_layer * g.nz;
  const int KW = TM + 2 * g.bx;
  // K-chunks: the window split into equal chunks of at most 128 rows (multiples of 4)
  const int nch = (KW + 127) / 128;
  int KC = ((KW + nch - 1) / nch + 3) / 4 * 4;
  int MC = ((int)N + 3) / 4 * 4;
  const size_t budget = 72 * 1024;
  while (MC > 4 && smem_bytes<T, RB, SB>(g, KC, MC) > budget) MC -= 4;
  while (KC > 16 && smem_bytes<T, RB, SB>(g, KC, MC) > budget) KC -= 16;
  const size_t smem = smem_bytes<T, RB, SB>(g, KC, MC);
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  static std::atomic<bool> attr_set{false};  // once per instantiation: allow more than 64 KiB of dynamic LDS
  if (!attr_set.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cov_stencil<T, RB, SB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr_set.store(true, std::memory_order_release);
  }
  dim3 grid(ntiles, (unsigned)((B + NS - 1) / NS));
  hipLaunchKernelGGL((k_cov_stencil<T, RB, SB>), grid, dim3(256), smem, st, g, Z, ldz, (int)N, V, ldv, vcols, (int)B,
                     Bdev, Tout, ldt, tiles_per_layer, KC, MC, prof, zero_counter);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rb(int rows_per_wave, const Grid& g, const T* Z, int64_t ldz, int64_t N, const T* V, int64_t ldv,
                     int64_t vcols, int64_t B, const int32_t* Bdev, T* Tout, int64_t ldt, hipStream_t st,
                     const ProfDev& pf, int32_t* zc) {
  // rows_per_wave selects the tile: 16 -> 16 rows x 32 systems, 32 -> 32 x 32, 64 -> 64 x 16, 128 -> 64 x 32
  switch (rows_per_wave) {
    case 16: return launch_typed<T, 1, 2>(g, Z, ldz, N, V, ldv, vcols, B, Bdev, Tout, ldt, st, pf, zc);
    case 32: return launch_typed<T, 2, 2>(g, Z, ldz, N, V, ldv, vcols, B, Bdev, Tout, ldt, st, pf, zc);
    case 64: return launch_typed<T, 4, 1>(g, Z, ldz, N, V, ldv, vcols, B, Bdev, Tout, ldt, st, pf, zc);
    case 128: return launch_typed<T, 4, 2>(g, Z, ldz, N, V, ldv, vcols, B, Bdev, Tout, ldt, st, pf, zc);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// BF16 variant (FP32 accumulation).  The member-dependent factor goes into the A
// operand, A_i[r, k] = L[r, k] z_i[k] (rounded to BF16 once per fragment), and the
// B operand is the member-independent BF16 copy of V, so the B fragments are staged
// once per block and reused by every member:
//   T_i = A_i V (MFMA, FP32 accumulate),   out[r, b] += z_i[r] T_i[r, b]  (FP32 epilogue).
// V is stored system-major (column b contiguous in k) so a lane's eight consecutive
// k of one fragment are one aligned 16-byte LDS read.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kPadB = 48;  // a band-overlapping 16x32 fragment reads up to 46 entries past the band

template <int RB, int SB>
__global__ __launch_bounds__(256) void k_cov_bf16(Grid g, const float* __restrict__ Z, int64_t ldz, int N,
                                                  const __hip_bfloat16* __restrict__ V, int64_t ldk, int64_t vcols,
                                                  int B, const int32_t* __restrict__ Bdev, float* __restrict__ Tout,
                                                  int64_t ldt, int tiles_per_layer, int KWs, int MC, ProfDev prof,
                                                  int32_t* __restrict__ zero_counter) {
  constexpr int TM = 16 * RB;
  constexpr int NS = 16 * SB;
  if (Bdev) B = *Bdev;
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
    if (zero_counter) {  // list and live counters of the next PCG step (nobody reads them now)
      zero_counter[0] = 0;
      zero_counter[1] = 0;
    }
    if (prof.vectors) {
      atomicAdd(prof.vectors, (unsigned long long)B);
      atomicAdd(prof.flops, (double)B * prof.flops_per_vector);
      atomicAdd(prof.bytes, (double)B * prof.bytes_per_vector);
    }
  }
  const int b0 = blockIdx.y * NS;
  if (b0 >= B) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int bx = g.bx, bz = g.bz, nl = 2 * bz + 1;
  const int tw = 2 * bx + 1 + 2 * kPadB;
  float* tab = reinterpret_cast<float*>(smem_raw);                    // nl x tw
  const int tab_sz = (nl * tw + 3) / 4 * 4;
  __hip_bfloat16* Vs = reinterpret_cast<__hip_bfloat16*>(tab + tab_sz);  // nl x NS x KWs
  float* Zw = reinterpret_cast<float*>(Vs + (size_t)nl * NS * KWs);     // nl x MC x KWs
  float* Zr = Zw + (size_t)nl * MC * KWs;                               // MC x TM
  int* kxs = reinterpret_cast<int*>(Zr + MC * TM);                      // nl x KWs: source index, -1 outside
  const int tile = blockIdx.x;
  const int z = tile / tiles_per_layer;
  const int x0 = (tile % tiles_per_layer) * TM;
  const int nx = g.nx, nz = g.nz;
  const int KW = TM + 2 * bx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lrow = lane & 15, lk = lane >> 4;

  for (int t = threadIdx.x; t < nl * tw; t += blockDim.x) {
    const int row = t / tw, c = t % tw - kPadB;
    tab[t] = (c >= 0 && c <= 2 * bx) ? g.table32[row * (2 * bx + 1) + c] : 0.f;
  }
  // source state index (layer offset + wrapped x) of every window position of every stencil layer
  for (int li = 0; li < nl; ++li)
    for (int kw = threadIdx.x; kw < KWs; kw += blockDim.x) {
      int zz = z + li - bz;
      bool ok = kw < KW;
      if (g.pz) zz = wrap_mod(zz, nz);
      else ok = ok && zz >= 0 && zz < nz;
      int kx = x0 - bx + kw;
      if (g.px) kx = wrap_mod(kx, nx);
      else ok = ok && kx >= 0 && kx < nx;
      kxs[li * KWs + kw] = ok ? zz * nx + kx : -1;
    }
  __syncthreads();
  // member-independent B operand: BF16 V window of every stencil layer (a wavefront per column)
  for (int r = wave; r < nl * NS; r += 4) {
    const int li = r / NS, bl = r % NS;
    const bool colok = (b0 + bl) < vcols;
    const __hip_bfloat16* vcol = V + (int64_t)(b0 + bl) * ldk;
    const int* ks = kxs + li * KWs;
    __hip_bfloat16* dst = Vs + (size_t)r * KWs;
    for (int kw = lane; kw < KWs; kw += 64) {
      const int k = ks[kw];
      dst[kw] = (colok && k >= 0) ? vcol[k] : __float2bfloat16(0.f);
    }
  }

  f4v out[RB][SB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) out[rb][sb] = f4v{0.f, 0.f, 0.f, 0.f};
  const int nK = KWs / 32;

  for (int m0 = 0; m0 < N; m0 += MC) {
    const int mcn = min(MC, N - m0);
    __syncthreads();
    for (int r = wave; r < nl * MC; r += 4) {
      const int li = r / MC, j = r % MC;
      const bool jok = j < mcn;
      const float* zcol = Z + (int64_t)(m0 + (jok ? j : 0)) * ldz;
      const int* ks = kxs + li * KWs;
      float* dst = Zw + (size_t)r * KWs;
      for (int kw = lane; kw < KWs; kw += 64) {
        const int k = ks[kw];
        dst[kw] = (jok && k >= 0) ? zcol[k] : 0.f;
      }
    }
    for (int t = threadIdx.x; t < MC * TM; t += blockDim.x) {
      const int j = t / TM, r = t % TM;
      Zr[t] = (j < mcn && x0 + r < nx) ? Z[(int64_t)(m0 + j) * ldz + (int64_t)z * nx + x0 + r] : 0.f;
    }
    __syncthreads();
    for (int j = wave; j < mcn; j += 4) {
      f4v acc[RB][SB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int sb = 0; sb < SB; ++sb) acc[rb][sb] = f4v{0.f, 0.f, 0.f, 0.f};
      for (int li = 0; li < nl; ++li) {
        const int zz = z + li - bz;
        if (!g.pz && (zz < 0 || zz >= nz)) continue;
        const float* trow = tab + li * tw + kPadB;
        const float* zrow = Zw + ((size_t)li * MC + j) * KWs;
        const __hip_bfloat16* vrow = Vs + (size_t)li * NS * KWs;
        for (int kk = 0; kk < nK; ++kk) {
          const int kb = 32 * kk + 8 * lk;
          const f4v za = *reinterpret_cast<const f4v*>(zrow + kb);
          const f4v zb = *reinterpret_cast<const f4v*>(zrow + kb + 4);
          bf8 bv[SB];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb)
            bv[sb] = *reinterpret_cast<const bf8*>(vrow + (size_t)(16 * sb + lrow) * KWs + kb);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            const int base = 32 * kk - 16 * rb;
            if (base + 31 >= 0 && base - 15 <= 2 * bx) {
              const int d0 = base + 8 * lk - lrow;
              bf8 a;
              a[0] = (__bf16)(trow[d0 + 0] * za[0]);
              a[1] = (__bf16)(trow[d0 + 1] * za[1]);
              a[2] = (__bf16)(trow[d0 + 2] * za[2]);
              a[3] = (__bf16)(trow[d0 + 3] * za[3]);
              a[4] = (__bf16)(trow[d0 + 4] * zb[0]);
              a[5] = (__bf16)(trow[d0 + 5] * zb[1]);
              a[6] = (__bf16)(trow[d0 + 6] * zb[2]);
              a[7] = (__bf16)(trow[d0 + 7] * zb[3]);
#pragma unroll
              for (int sb = 0; sb < SB; ++sb)
                acc[rb][sb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bv[sb], acc[rb][sb], 0, 0, 0);
            }
          }
        }
      }
      // epilogue: out[r, b] += z_j[r] T_j[r, b]; D register v of lane l is row 4(l/16) + v
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float zr = Zr[j * TM + 16 * rb + 4 * lk + v];
#pragma unroll
          for (int sb = 0; sb < SB; ++sb) out[rb][sb][v] += zr * acc[rb][sb][v];
        }
    }
  }

  __syncthreads();
  float* red = reinterpret_cast<float*>(smem_raw);
  constexpr int PER = RB * SB * 4;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[((wave * PER) + (rb * SB + sb) * 4 + v) * 64 + lane] = out[rb][sb][v];
  __syncthreads();
  for (int f = wave; f < RB * SB; f += 4) {
    const int rb = f / SB, sb = f % SB;
    const int b = b0 + 16 * sb + lrow;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      float sacc = 0.f;
#pragma unroll
      for (int w = 0; w < 4; ++w) sacc += red[((w * PER) + f * 4 + v) * 64 + lane];
      const int x = x0 + 16 * rb + 4 * lk + v;
      if (x < nx && b < B) Tout[(int64_t)b * ldt + (int64_t)z * nx + x] = sacc;
    }
  }
}

template <int RB, int SB>
size_t smem_bf16(const Grid& g, int KWs, int MC) {
  constexpr int TM = 16 * RB, NS = 16 * SB;
  const int nl = 2 * g.bz + 1;
  const size_t tab = (size_t)((nl * (2 * g.bx + 1 + 2 * kPadB) + 3) / 4 * 4) * 4;
  const size_t stage = tab + (size_t)nl * NS * KWs * 2 + (size_t)nl * MC * KWs * 4 + (size_t)MC * TM * 4 +
                       (size_t)nl * KWs * 4;
  const size_t red = (size_t)4 * 64 * RB * SB * 4 * 4;
  return stage > red ? stage : red;
}

template <int RB, int SB>
hipError_t launch_bf16_typed(const Grid& g, const float* Z, int64_t ldz, int64_t N, const __hip_bfloat16* V,
                             int64_t ldk, int64_t vcols, int64_t B, const int32_t* Bdev, float* T, int64_t ldt,
                             hipStream_t st, const ProfDev& prof, int32_t* zero_counter) {
  constexpr int TM = 16 * RB, NS = 16 * SB;
  const int tiles_per_layer = (g.nx + TM - 1) / TM;
  const int ntiles = tiles_per_layer * g.nz;
  const int KWs = (TM + 2 * g.bx + 31) / 32 * 32;
  int MC = ((int)N + 3) / 4 * 4;
  const size_t budget = 96 * 1024;
  while (MC > 4 && smem_bf16<RB, SB>(g, KWs, MC) > budget) MC -= 4;
  const size_t smem = smem_bf16<RB, SB>(g, KWs, MC);
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  static std::atomic<bool> attr{false};  // concurrent first calls set the same attribute twice: harmless
  if (!attr.load(std::memory_order_acquire)) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cov_bf16<RB, SB>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
  }
  dim3 grid(ntiles, (unsigned)((B + NS - 1) / NS));
  hipLaunchKernelGGL((k_cov_bf16<RB, SB>), grid, dim3(256), smem, st, g, Z, ldz, (int)N, V, ldk, vcols, (int)B, Bdev,
                     T, ldt, tiles_per_layer, KWs, MC, prof, zero_counter);
  return hipGetLastError();
}

// Dense L (small n, tests): T[r, b] = sum_i z_i[r] sum_k L[r,k] z_i[k] V[k,b]; one thread per (r, b);
// V and T system-major.
__global__ void k_cov_dense(const double* __restrict__ L, const double* __restrict__ Z, int64_t n, int64_t N,
                            const double* __restrict__ V, int64_t ldv, int64_t B, double* __restrict__ T,
                            int64_t ldt) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * B) return;
  const int64_t r = t / B, b = t % B;
  double acc = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    double inner = 0.0;
    for (int64_t k = 0; k < n; ++k) inner += L[r + k * n] * Z[k + i * n] * V[b * ldv + k];
    acc += Z[r + i * n] * inner;
  }
  T[b * ldt + r] = acc;
}

}  // namespace

hipError_t launch_cov_stencil(Prec prec, const Grid& g, const void* Z, int64_t ldz, int64_t N, const void* V,
                              int64_t ldv, int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt,
                              int rows_per_wave, hipStream_t st, const ProfDev* prof, int32_t* zero_counter) {
  if (B <= 0) return hipSuccess;
  if (!Z || !V || !T || (prec == Prec::F64 ? !g.table : !g.table32)) return hipErrorInvalidValue;
  const ProfDev pf = prof ? *prof : ProfDev{};
  switch (prec) {
    case Prec::F64:
      return launch_rb<double>(rows_per_wave, g, (const double*)Z, ldz, N, (const double*)V, ldv, vcols, B, Bdev,
                               (double*)T, ldt, st, pf, zero_counter);
    case Prec::F32:
      return launch_rb<float>(rows_per_wave, g, (const float*)Z, ldz, N, (const float*)V, ldv, vcols, B, Bdev,
                              (float*)T, ldt, st, pf, zero_counter);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cov_bf16(const Grid& g, const float* Z, int64_t ldz, int64_t N, const __hip_bfloat16* V,
                           int64_t ldk, int64_t vcols, int64_t B, const int32_t* Bdev, float* T, int64_t ldt, int tile,
                           hipStream_t st, const ProfDev* prof, int32_t* zc) {
  if (B <= 0) return hipSuccess;
  if (!Z || !V || !T || !g.table32) return hipErrorInvalidValue;
  const ProfDev pf = prof ? *prof : ProfDev{};
  switch (tile) {
    case 16: return launch_bf16_typed<1, 2>(g, Z, ldz, N, V, ldk, vcols, B, Bdev, T, ldt, st, pf, zc);
    case 32: return launch_bf16_typed<2, 2>(g, Z, ldz, N, V, ldk, vcols, B, Bdev, T, ldt, st, pf, zc);
    case 64: return launch_bf16_typed<1, 4>(g, Z, ldz, N, V, ldk, vcols, B, Bdev, T, ldt, st, pf, zc);
    case 128: return launch_bf16_typed<1, 8>(g, Z, ldz, N, V, ldk, vcols, B, Bdev, T, ldt, st, pf, zc);
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
