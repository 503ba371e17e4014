// Localized covariance held as an explicit band (Sec. 2.3, eq. 2.11).
//
// P = L o (Z Z^T) has the sparsity of the stationary stencil L: row r couples only to the
// (2bz+1)(2bx+1) grid neighbours r + (dz, dx).  Its entries
//
//   band[j, r] = L(dz, dx) * sum_i Z[r, i] Z[r + (dz, dx), i],   j = (dz + bz)(2bx + 1) + (dx + bx)
//
// cost one pass over the members (N fused multiply-adds per entry, done once per update), after
// which an apply is a banded product, 2 nnz(L) flops per vector instead of the 2 N nnz(L) of the
// operator form sum_i z_i o L (z_i o v) (eq. 2.12).  The operator form stays the path for grids
// whose band does not fit in memory; both give P V up to rounding.
//
// Layout: band[j * ldb + r] (one plane per stencil offset, rows contiguous, so the lanes of a
// wavefront read consecutive rows of one plane).  Entries whose neighbour falls off a
// non-periodic grid are 0.
#include <atomic>

#include "internal.hpp"

namespace infoesrf {

namespace {

__device__ inline int wrap_idx(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

template <typename T>
__global__ __launch_bounds__(256) void k_band_build(Grid g, const double* __restrict__ Z, int64_t ldz, int N,
                                                    T* __restrict__ band, int64_t ldb) {
  const int rows = g.nz * g.nx;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (r >= rows) return;
  const int w = 2 * g.bx + 1;
  const int dz = j / w - g.bz, dx = j % w - g.bx;
  const int z = r / g.nx, x = r % g.nx;
  int zz = z + dz, xx = x + dx;
  bool ok = true;
  if (g.pz) zz = wrap_idx(zz, g.nz);
  else ok = ok && zz >= 0 && zz < g.nz;
  if (g.px) xx = wrap_idx(xx, g.nx);
  else ok = ok && xx >= 0 && xx < g.nx;
  double v = 0.0;
  const double l = g.table[j];
  if (ok && l != 0.0) {
    const int64_t c = (int64_t)zz * g.nx + xx;
    double s = 0.0;
    for (int i = 0; i < N; ++i) s = fma(Z[(int64_t)i * ldz + r], Z[(int64_t)i * ldz + c], s);
    v = l * s;
  }
  band[(int64_t)j * ldb + r] = (T)v;
}

// The same entries on MFMA.  For a tile of 16 consecutive lattice points (z, x0 .. x0 + 15) and
// one stencil row li, the dot products of their member rows Z[r, :] with those of the 16 + 2bx
// points (z + li - bz, x0 - bx ..) of the neighbour layer are a 16 x (16 + 2bx) block of Z Z^T
// (contraction over the N members), formed 16 columns at a time by v_mfma_f64_16x16x4f64 (the
// block's four wavefronts take every fourth column tile).  The products on the band,
// d = c - r + bx in [0, 2bx], go to an LDS tile [d][row], written out plane by plane (16
// consecutive rows, 128 bytes) times the table weight.  Neighbours off a non-periodic grid enter
// as zero rows of Z, so their entries are 0.  N <= 64 (the A fragments stay in registers) and
// 16 (2bx + 1) doubles of LDS.
typedef double band_d4 __attribute__((ext_vector_type(4)));
constexpr int kBuildMaxN = 64;
constexpr int kBuildMaxW = 511;

template <typename T>
__global__ __launch_bounds__(256) void k_band_build_mfma(Grid g, const double* __restrict__ Z, int64_t ldz, int N,
                                                         T* __restrict__ band, int64_t ldb, int tiles_per_layer) {
  extern __shared__ double btile[];  // [w][16]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int w = 2 * g.bx + 1;
  const int li = blockIdx.y;
  const int z = blockIdx.x / tiles_per_layer;
  const int x0 = (blockIdx.x % tiles_per_layer) * 16;
  int zz = z + li - g.bz;
  bool zok = true;
  if (g.pz) zz = wrap_idx(zz, g.nz);
  else zok = zz >= 0 && zz < g.nz;
  // v_mfma_f64_16x16x4f64: A lane l -> (row l%16, k l/16); B lane l -> (k l/16, col l%16);
  // D register v of lane l -> (row 4v + l/16, col l%16)
  const int i = lane & 15, kq = lane >> 4;
  const int KS = (N + 3) / 4;
  const bool rok = x0 + i < g.nx;
  const int64_t r = (int64_t)z * g.nx + x0 + i;
  double a[kBuildMaxN / 4];
#pragma unroll
  for (int ks = 0; ks < kBuildMaxN / 4; ++ks) {
    const int k = 4 * ks + kq;
    a[ks] = (k < N && rok) ? Z[(int64_t)k * ldz + r] : 0.0;
  }
  const int nct = (16 + 2 * g.bx + 15) / 16;
  for (int ct = wave; ct < nct; ct += 4) {
    int xc = x0 - g.bx + 16 * ct + i;
    bool cok = zok;
    if (g.px) xc = wrap_idx(xc, g.nx);
    else cok = cok && xc >= 0 && xc < g.nx;
    const int64_t c = (int64_t)zz * g.nx + xc;
    double b[kBuildMaxN / 4];
#pragma unroll
    for (int ks = 0; ks < kBuildMaxN / 4; ++ks) {
      const int k = 4 * ks + kq;
      b[ks] = (ks < KS && k < N && cok) ? Z[(int64_t)k * ldz + c] : 0.0;
    }
    band_d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < kBuildMaxN / 4; ++ks)
      if (ks < KS) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + kq;
      const int d = 16 * ct + i - row;
      if (d >= 0 && d < w) btile[d * 16 + row] = acc[v];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < w * 16; t += 256) {
    const int d = t >> 4, row = t & 15;
    if (x0 + row < g.nx) {
      const double l = g.table[li * w + d];
      band[(int64_t)(li * w + d) * ldb + (int64_t)z * g.nx + x0 + row] = (T)(l * btile[t]);
    }
  }
}

// T[:, b] = band * V[:, b] for the listed columns b < B (B from Bdev when given).
// Block: TX = 64 consecutive x of one layer (one lane each) x NSB systems (the four waves take
// systems w, w + 4, ...).  For each stencil layer the block stages the V window
// [x0 - bx, x0 + 64 + bx) of its systems in LDS; every lane then runs over the 2bx + 1 offsets,
// loading each band entry once (eight at a time, so the loads overlap) and using it for its
// NSB / 4 systems.
template <typename T, int NSB>
__global__ __launch_bounds__(256) void k_band_apply(Grid g, const T* __restrict__ band, int64_t ldb,
                                                    const T* __restrict__ V, int64_t ldv, int64_t vcols, int B,
                                                    const int32_t* __restrict__ Bdev, T* __restrict__ Tout,
                                                    int64_t ldt, int tiles_per_layer, ProfDev prof,
                                                    int32_t* __restrict__ zero_counter) {
  constexpr int TX = 64;
  constexpr int PER = NSB / 4;
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
  const int b0 = blockIdx.y * NSB;
  if (b0 >= B) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  T* Vw = reinterpret_cast<T*>(smem_raw);  // NSB x WX
  const int nx = g.nx, nz = g.nz, bx = g.bx, bz = g.bz;
  const int WX = TX + 2 * bx;
  const int tile = blockIdx.x;
  const int z = tile / tiles_per_layer;
  const int x0 = (tile % tiles_per_layer) * TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = x0 + lane;
  const bool row_ok = x < nx;
  const int64_t r = (int64_t)z * nx + x;
  const int w = 2 * bx + 1;

  T acc[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) acc[k] = T(0);

  for (int li = 0; li < 2 * bz + 1; ++li) {
    int zz = z + li - bz;
    if (g.pz) zz = wrap_idx(zz, nz);
    else if (zz < 0 || zz >= nz) continue;  // uniform over the block
    __syncthreads();
    // each lane stages window positions t = lane, lane + 64, ... of the wave's PER columns; the
    // PER loads of one position are independent, so they are in flight together
    const T* vbase = V + (int64_t)zz * nx;
    for (int t = lane; t < WX; t += 64) {
      int kx = x0 - bx + t;
      bool ok = true;
      if (g.px) kx = wrap_idx(kx, nx);
      else ok = kx >= 0 && kx < nx;
      T v[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int c = wave + 4 * k;
        v[k] = (ok && b0 + c < vcols) ? vbase[(int64_t)(b0 + c) * ldv + kx] : T(0);  // no column past vcols
      }
#pragma unroll
      for (int k = 0; k < PER; ++k) Vw[(wave + 4 * k) * WX + t] = v[k];
    }
    __syncthreads();
    if (row_ok) {
      const T* bp = band + (int64_t)(li * w) * ldb + r;
      const T* vw = Vw + wave * WX + lane;
      int d = 0;
      for (; d + 8 <= w; d += 8) {
        T bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bv[u] = bp[(int64_t)(d + u) * ldb];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int k = 0; k < PER; ++k) acc[k] = fma(bv[u], vw[4 * k * WX + d + u], acc[k]);
      }
      for (; d < w; ++d) {
        const T bv = bp[(int64_t)d * ldb];
#pragma unroll
        for (int k = 0; k < PER; ++k) acc[k] = fma(bv, vw[4 * k * WX + d], acc[k]);
      }
    }
  }
  if (row_ok) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int b = b0 + wave + 4 * k;
      if (b < B) Tout[(int64_t)b * ldt + r] = acc[k];
    }
  }
}

template <typename T, int NSB>
hipError_t band_apply_typed(const Grid& g, const T* band, int64_t ldb, const T* V, int64_t ldv, int64_t vcols,
                            int64_t B, const int32_t* Bdev, T* Tout, int64_t ldt, hipStream_t st, const ProfDev& pf,
                            int32_t* zc) {
  constexpr int TX = 64;
  const int tiles_per_layer = (g.nx + TX - 1) / TX;
  const size_t smem = sizeof(T) * (size_t)NSB * (TX + 2 * g.bx);
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  static std::atomic<bool> attr{false};  // concurrent first calls set the same attribute twice: harmless
  if (smem > 64 * 1024 && !attr.load(std::memory_order_acquire)) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_band_apply<T, NSB>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    attr.store(true, std::memory_order_release);
  }
  dim3 grid((unsigned)(tiles_per_layer * g.nz), (unsigned)((B + NSB - 1) / NSB));
  hipLaunchKernelGGL((k_band_apply<T, NSB>), grid, dim3(256), smem, st, g, band, ldb, V, ldv, vcols, (int)B, Bdev,
                     Tout, ldt, tiles_per_layer, pf, zc);
  return hipGetLastError();
}

}  // namespace

static int band_systems_per_block(const Grid& g, size_t elem, int64_t B) {
  // a measured choice for this grid and batch size (infoesrf_autotune), if it fits in LDS
  // (halved while half of it still holds the batch: wider blocks would only add zero columns, and
  // a bucket's choice is measured at a larger batch than its smallest)
  int t = tuned_choice(TuneKey{0, elem == 8 ? 0 : 1, g.nz, g.nx, g.bz, g.bx, 0}, B);
  while (t > 8 && t / 2 >= B) t /= 2;
  if ((t == 8 || t == 16 || t == 32 || t == 64) && (size_t)t * (64 + 2 * g.bx) * elem <= 150 * 1024) return t;
  // else the widest system block whose V window stays within 48 KiB of LDS (four blocks per CU),
  // and no wider than the batch needs
  for (int nsb : {64, 32, 16}) {
    if ((size_t)nsb * (64 + 2 * g.bx) * elem <= 48 * 1024 && (nsb <= 16 || B > nsb / 2)) return nsb;
  }
  return 8;
}

hipError_t launch_band_build(Prec prec, const Grid& g, const double* Z, int64_t ldz, int64_t N, void* band,
                             int64_t ldb, hipStream_t st) {
  const int rows = g.nz * g.nx;
  const int nb = (2 * g.bz + 1) * (2 * g.bx + 1);
  if (!band || !Z || !g.table) return hipErrorInvalidValue;
  const int w = 2 * g.bx + 1;
  if (N <= kBuildMaxN && w <= kBuildMaxW) {
    const int tpl = (g.nx + 15) / 16;
    const dim3 grid((unsigned)(g.nz * tpl), (unsigned)(2 * g.bz + 1));
    const size_t lds = (size_t)w * 16 * sizeof(double);
    if (prec == Prec::F64)
      hipLaunchKernelGGL((k_band_build_mfma<double>), grid, dim3(256), lds, st, g, Z, ldz, (int)N, (double*)band,
                         ldb, tpl);
    else
      hipLaunchKernelGGL((k_band_build_mfma<float>), grid, dim3(256), lds, st, g, Z, ldz, (int)N, (float*)band, ldb,
                         tpl);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((rows + 255) / 256), (unsigned)nb);
  if (prec == Prec::F64)
    hipLaunchKernelGGL((k_band_build<double>), grid, dim3(256), 0, st, g, Z, ldz, (int)N, (double*)band, ldb);
  else
    hipLaunchKernelGGL((k_band_build<float>), grid, dim3(256), 0, st, g, Z, ldz, (int)N, (float*)band, ldb);
  return hipGetLastError();
}

hipError_t launch_band_apply(Prec prec, const Grid& g, const void* band, int64_t ldb, const void* V, int64_t ldv,
                             int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt, hipStream_t st,
                             const ProfDev* prof, int32_t* zc) {
  if (B <= 0) return hipSuccess;
  if (!band || !V || !T) return hipErrorInvalidValue;
  const ProfDev pf = prof ? *prof : ProfDev{};
  if (prec == Prec::F64) {
    const double* b = (const double*)band;
    const double* v = (const double*)V;
    double* t = (double*)T;
    switch (band_systems_per_block(g, sizeof(double), B)) {
      case 64: return band_apply_typed<double, 64>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
      case 32: return band_apply_typed<double, 32>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
      case 16: return band_apply_typed<double, 16>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
      default: return band_apply_typed<double, 8>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
    }
  }
  if (prec == Prec::F32) {
    const float* b = (const float*)band;
    const float* v = (const float*)V;
    float* t = (float*)T;
    switch (band_systems_per_block(g, sizeof(float), B)) {
      case 64: return band_apply_typed<float, 64>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
      case 32: return band_apply_typed<float, 32>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
      case 16: return band_apply_typed<float, 16>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
      default: return band_apply_typed<float, 8>(g, b, ldb, v, ldv, vcols, B, Bdev, t, ldt, st, pf, zc);
    }
  }
  return hipErrorInvalidValue;  // the band form has FP64 and FP32 entries only
}

// ---------------------------------------------------------------- rectangular state x lattice band
namespace {

constexpr int kRectTX = 64;  // state points of one grid row a block takes

__host__ __device__ inline int rect_floor_div(int p, int q) { return p >= 0 ? p / q : -((-p + q - 1) / q); }
__host__ __device__ inline int rect_ceil_div(int p, int q) { return -rect_floor_div(-p, q); }
__device__ inline int rect_wrap(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}
// Lattice columns a block's window spans: those of its first point's window up to its last
// point's (at most (TX - 1) / sx + 1 more than one point's wx).
__host__ __device__ inline int rect_window_cols(const RectGeom& g) { return (kRectTX - 1) / g.sx + 1 + g.wx; }

// The block's tile and window: grid row z, first column x0, nxt points; the window's first
// lattice row a0 and column b0 and its nb columns.
struct RectTile {
  int z, x0, nxt, a0, b0, nb;
};
__device__ inline RectTile rect_tile(const RectGeom& g, int tiles_per_row) {
  RectTile t;
  t.z = blockIdx.x / tiles_per_row;
  t.x0 = (blockIdx.x % tiles_per_row) * kRectTX;
  t.nxt = min(kRectTX, g.nx - t.x0);
  t.a0 = rect_ceil_div(t.z - g.bz - g.z0, g.sz);
  t.b0 = rect_ceil_div(t.x0 - g.bx - g.x0, g.sx);
  t.nb = rect_ceil_div(t.x0 + t.nxt - 1 - g.bx - g.x0, g.sx) + g.wx - t.b0;
  return t;
}
// Row-major lattice index of window point (ia, ib), or -1 past a lattice end that is not periodic.
__device__ inline int rect_window_point(const RectGeom& g, const RectTile& t, int ia, int ib) {
  int a = t.a0 + ia, b = t.b0 + ib;
  if (g.pz) a = rect_wrap(a, g.nzo);
  else if (a < 0 || a >= g.nzo) return -1;
  if (g.px) b = rect_wrap(b, g.nxo);
  else if (b < 0 || b >= g.nxo) return -1;
  return a * g.nxo + b;
}

// One block per (tile, chunk of kRectEB entries): Z of its points and the lattice members of its
// window staged in LDS, then R[e ldr + j] = L(dz, dx) sum_i Z[j, i] Zt[k, i] for the chunk's
// entries e = ia wx + ib of every point j (zero where the lattice point lies outside the point's
// window or past a lattice end); four independent chains over the members.
constexpr int kRectEB = 16;
__global__ __launch_bounds__(256) void k_rect_build(RectGeom g, const double* __restrict__ Z, int64_t ldz,
                                                     const double* __restrict__ Zt, int64_t ldzt, int N,
                                                     double* __restrict__ R, int64_t ldr, int tiles_per_row) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  const RectTile t = rect_tile(g, tiles_per_row);
  const int tid = threadIdx.x;
  const int nw = g.wz * t.nb;
  double* Zs = sm;                   // N x kRectTX
  double* Ws = sm + N * kRectTX;     // N x nw
  const int64_t row0 = (int64_t)t.z * g.nx + t.x0;
  // a point (or window point) a thread and its members in batches of 8 loads ahead of their
  // stores (a store right after each load would wait for every load in turn)
  constexpr int LB = 8;
  for (int xx = tid; xx < kRectTX * 4; xx += 256) {
    const int p = xx & (kRectTX - 1), i0 = xx / kRectTX;
    if (p >= t.nxt) continue;
    for (int ib = i0; ib < N; ib += 4 * LB) {
      double v[LB];
#pragma unroll
      for (int h = 0; h < LB; ++h) v[h] = ib + 4 * h < N ? Z[(ib + 4 * h) * ldz + row0 + p] : 0.0;
#pragma unroll
      for (int h = 0; h < LB; ++h)
        if (ib + 4 * h < N) Zs[(ib + 4 * h) * kRectTX + p] = v[h];
    }
  }
  for (int v = tid; v < nw; v += 256) {
    const int k = rect_window_point(g, t, v / t.nb, v % t.nb);
    for (int ib = 0; ib < N; ib += LB) {
      double w[LB];
#pragma unroll
      for (int h = 0; h < LB; ++h) w[h] = (k >= 0 && ib + h < N) ? Zt[(ib + h) * ldzt + k] : 0.0;
#pragma unroll
      for (int h = 0; h < LB; ++h)
        if (ib + h < N) Ws[(ib + h) * nw + v] = w[h];
    }
  }
  __syncthreads();
  const int W = g.wz * g.wx, wt = 2 * g.bx + 1;
  const int e0 = blockIdx.y * kRectEB, e1 = min(W, e0 + kRectEB);
  for (int u = tid; u < (e1 - e0) * kRectTX; u += 256) {
    const int e = e0 + u / kRectTX, xx = u % kRectTX;  // consecutive threads take consecutive points
    if (xx >= t.nxt) continue;
    const int x = t.x0 + xx, ia = e / g.wx, ib = e % g.wx;
    const int blo = rect_ceil_div(x - g.bx - g.x0, g.sx);
    const int dz = g.z0 + g.sz * (t.a0 + ia) - t.z, dx = g.x0 + g.sx * (blo + ib) - x;
    double val = 0.0;
    if (dz <= g.bz && dx <= g.bx) {
      const int v = ia * t.nb + (blo - t.b0) + ib;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int i = 0;
      for (; i + 4 <= N; i += 4) {
#pragma unroll
        for (int h = 0; h < 4; ++h) acc[h] += Zs[(i + h) * kRectTX + xx] * Ws[(i + h) * nw + v];
      }
      for (; i < N; ++i) acc[0] += Zs[i * kRectTX + xx] * Ws[i * nw + v];
      val = g.table[(dz + g.bz) * wt + dx + g.bx] * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
    R[(int64_t)e * ldr + row0 + xx] = val;
  }
}

// One block per (tile, group of 4 CPT columns): the window's entries of those listed columns of U
// staged in LDS, then wavefront w takes the tile's 64 points for columns w, w + 4, ... of the
// group; the band entries go in batches of 8 loads ahead of their use.
template <int CPT>
__global__ __launch_bounds__(256) void k_rect_apply(RectGeom g, const double* __restrict__ R, int64_t ldr,
                                                     const double* __restrict__ U, int64_t ldu,
                                                     const int32_t* __restrict__ act, const int32_t* __restrict__ nact,
                                                     int ncols, double* __restrict__ T, int64_t ldt,
                                                     int tiles_per_row) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  const RectTile t = rect_tile(g, tiles_per_row);
  const int tid = threadIdx.x;
  const int nw = g.wz * t.nb;
  const int na = nact ? min(*nact, ncols) : ncols;
  const int cb = blockIdx.y * 4 * CPT;  // the group's first column
  const int nc = min(4 * CPT, na - cb);
  if (nc <= 0) return;
  for (int v = tid; v < nw; v += 256) {
    const int k = rect_window_point(g, t, v / t.nb, v % t.nb);
    double w[4 * CPT];
#pragma unroll
    for (int c = 0; c < 4 * CPT; ++c) w[c] = (k >= 0 && c < nc) ? U[(int64_t)act[cb + c] * ldu + k] : 0.0;
#pragma unroll
    for (int c = 0; c < 4 * CPT; ++c)
      if (c < nc) sm[c * nw + v] = w[c];
  }
  __syncthreads();
  const int xx = tid & 63, grp = tid >> 6;
  if (xx >= t.nxt) return;
  const int x = t.x0 + xx;
  const int64_t j = (int64_t)t.z * g.nx + x;
  const int boff = rect_ceil_div(x - g.bx - g.x0, g.sx) - t.b0;
  double acc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) acc[q] = 0.0;
  constexpr int EB = 8;
  for (int ia = 0; ia < g.wz; ++ia) {
    const double* rrow = R + (int64_t)(ia * g.wx) * ldr + j;  // zero outside the point's window
    const double* srow = sm + ia * t.nb + boff;
    int ib = 0;
    for (; ib + EB <= g.wx; ib += EB) {
      double r[EB];
#pragma unroll
      for (int u = 0; u < EB; ++u) r[u] = rrow[(int64_t)(ib + u) * ldr];
#pragma unroll
      for (int u = 0; u < EB; ++u)
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          const int c = grp + 4 * q;
          if (c < nc) acc[q] += r[u] * srow[c * nw + ib + u];
        }
    }
    for (; ib < g.wx; ++ib) {
      const double r = rrow[(int64_t)ib * ldr];
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int c = grp + 4 * q;
        if (c < nc) acc[q] += r * srow[c * nw + ib];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int c = grp + 4 * q;
    if (c < nc) T[(int64_t)(cb + c) * ldt + j] = acc[q];
  }
}

size_t rect_build_lds(const RectGeom& g, int64_t N) {
  return sizeof(double) * (size_t)N * (kRectTX + (size_t)g.wz * rect_window_cols(g));
}
constexpr int kRectCPT = 2;  // columns a thread accumulates in the apply (8 a block)
size_t rect_apply_lds(const RectGeom& g, int64_t ncols) {
  return sizeof(double) * (size_t)std::min<int64_t>(ncols, 4 * kRectCPT) * g.wz * rect_window_cols(g);
}

}  // namespace

bool rect_fits(const Grid& gs, const infoesrf_lattice& lat, int64_t N) {
  if (lat.sz < 1 || lat.sx < 1 || lat.nzo < 1 || lat.nxo < 1) return false;
  if (gs.pz && (int64_t)lat.nzo * lat.sz != gs.nz) return false;
  if (gs.px && (int64_t)lat.nxo * lat.sx != gs.nx) return false;
  const RectGeom g = rect_geom(gs, lat);
  // the final apply takes N + 1 columns at most (members and the mean)
  return rect_build_lds(g, N) <= 64 * 1024 && rect_apply_lds(g, N + 1) <= 64 * 1024;
}

RectGeom rect_geom(const Grid& gs, const infoesrf_lattice& lat) {
  RectGeom g{};
  g.nz = gs.nz;
  g.nx = gs.nx;
  g.pz = gs.pz;
  g.px = gs.px;
  g.bz = gs.bz;
  g.bx = gs.bx;
  g.z0 = lat.z0;
  g.sz = lat.sz;
  g.nzo = lat.nzo;
  g.x0 = lat.x0;
  g.sx = lat.sx;
  g.nxo = lat.nxo;
  g.wz = 2 * gs.bz / lat.sz + 1;
  g.wx = 2 * gs.bx / lat.sx + 1;
  g.table = gs.table;
  return g;
}

hipError_t launch_rect_build(const RectGeom& g, const double* Z, int64_t ldz, const double* Zt, int64_t ldzt,
                             int64_t N, double* R, int64_t ldr, hipStream_t st) {
  const int64_t n = (int64_t)g.nz * g.nx;
  const size_t lds = rect_build_lds(g, N);
  if (!Z || !Zt || !R || !g.table || ldr < n || N < 1 || lds > 64 * 1024) return hipErrorInvalidValue;
  const int tpr = (g.nx + kRectTX - 1) / kRectTX;
  const int chunks = (g.wz * g.wx + kRectEB - 1) / kRectEB;
  hipLaunchKernelGGL(k_rect_build, dim3((unsigned)(tpr * g.nz), (unsigned)chunks), dim3(256), lds, st, g, Z, ldz, Zt,
                     ldzt, (int)N, R, ldr, tpr);
  return hipGetLastError();
}

hipError_t launch_rect_apply(const RectGeom& g, const double* R, int64_t ldr, const double* U, int64_t ldu,
                             const int32_t* act, const int32_t* nact, int64_t ncols, double* T, int64_t ldt,
                             hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  const int64_t n = (int64_t)g.nz * g.nx;
  const size_t lds = rect_apply_lds(g, ncols);
  if (!R || !U || !act || !T || ldt < n || lds > 64 * 1024) return hipErrorInvalidValue;
  const int tpr = (g.nx + kRectTX - 1) / kRectTX;
  const int groups = (int)((ncols + 4 * kRectCPT - 1) / (4 * kRectCPT));
  hipLaunchKernelGGL((k_rect_apply<kRectCPT>), dim3((unsigned)(tpr * g.nz), (unsigned)groups), dim3(256), lds, st, g, R,
                     ldr, U, ldu, act, nact, (int)ncols, T, ldt, tpr);
  return hipGetLastError();
}

}  // namespace infoesrf
