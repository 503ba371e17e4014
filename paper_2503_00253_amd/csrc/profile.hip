// Measurement hooks: HIP events around covariance-apply launches and device-side
// counters of the vectors, algorithmic FLOPs and algorithmic bytes they process.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.hpp"

namespace infoesrf {

namespace {

constexpr int kSlots = INFOESRF_PROF_SLOTS;

struct Prof {
  bool on = false;
  uint32_t mask = ~0u;  // slots measured while on
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> ev_slot;    // slot of each pair
  size_t used = 0;
  double ms[kSlots] = {};
  int64_t launches[kSlots] = {};
  double host_bytes[kSlots] = {};      // per-launch bytes (band or Z reads), added on the host
  unsigned long long* dvec = nullptr;  // [kSlots]
  double* dflops = nullptr;            // [kSlots]
  double* dbytes = nullptr;            // [kSlots]
};

Prof g_prof;
std::mutex g_prof_mu;  // launches from several host threads (batched instances) share the pool
constexpr size_t kPairs = 2048;

// Nonzeros of L on grid g.  The table is copied to the host once per (table, grid) key while
// profiling, so steady-state timed launches do not synchronize; a table rewritten in place under
// the same key during one profiling session keeps its first count.
double grid_nnz(const Grid& g) {
  using Key = std::tuple<const void*, int, int, int, int, int, int>;
  static std::map<Key, double> cache;
  const Key key{g.table, g.nz, g.nx, g.bz, g.bx, g.pz, g.px};
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const int w = 2 * g.bx + 1, h = 2 * g.bz + 1;
  std::vector<double> t((size_t)w * h);
  if (hipMemcpy(t.data(), g.table, sizeof(double) * t.size(), hipMemcpyDeviceToHost) != hipSuccess) return 0.0;
  double nnz = 0.0;
  for (int dz = -g.bz; dz <= g.bz; ++dz)
    for (int dx = -g.bx; dx <= g.bx; ++dx) {
      if (t[(size_t)(dz + g.bz) * w + (dx + g.bx)] == 0.0) continue;
      const double cz = g.pz ? g.nz : (double)std::max(0, g.nz - std::abs(dz));
      const double cx = g.px ? g.nx : (double)std::max(0, g.nx - std::abs(dx));
      nnz += cz * cx;
    }
  cache.emplace(key, nnz);
  return nnz;
}

hipError_t drain() {
  for (size_t i = 0; i < g_prof.used; ++i) {
    hipError_t e = hipEventSynchronize(g_prof.ev[2 * i + 1]);
    if (e != hipSuccess) return e;
    float t = 0.f;
    e = hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]);
    if (e != hipSuccess) return e;
    g_prof.ms[g_prof.ev_slot[i]] += t;
  }
  g_prof.used = 0;
  return hipSuccess;
}

// Brackets launch() with an event pair and fills the device counters of `slot`.
template <typename F>
hipError_t timed(int slot, double flops_per_vector, double bytes_per_vector, double bytes_per_launch,
                 hipStream_t st, F&& launch) {
  std::lock_guard<std::mutex> lock(g_prof_mu);
  if (!(g_prof.mask & (1u << slot))) return launch(nullptr);
  hipError_t e;
  if (g_prof.used == kPairs && (e = drain()) != hipSuccess) return e;
  ProfDev pd{g_prof.dvec + slot, g_prof.dflops + slot, flops_per_vector, g_prof.dbytes + slot, bytes_per_vector};
  const size_t k = g_prof.used++;
  g_prof.ev_slot[k] = slot;
  if ((e = hipEventRecord(g_prof.ev[2 * k], st)) != hipSuccess) return e;
  if ((e = launch(&pd)) != hipSuccess) return e;
  g_prof.launches[slot] += 1;
  g_prof.host_bytes[slot] += bytes_per_launch;
  return hipEventRecord(g_prof.ev[2 * k + 1], st);
}

size_t elem_size(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }

}  // namespace

hipError_t cov_stencil_timed(Prec prec, const Grid& g, const void* Z, int64_t ldz, int64_t N, const void* V,
                             int64_t ldv, int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt,
                             int rows_per_wave, hipStream_t st, int32_t* zc) {
  if (!g_prof.on)
    return launch_cov_stencil(prec, g, Z, ldz, N, V, ldv, vcols, B, Bdev, T, ldt, rows_per_wave, st, nullptr, zc);
  const double rows = (double)g.nz * g.nx;
  const double es = (double)elem_size(prec);
  return timed((int)prec, 2.0 * (double)N * grid_nnz(g) + 3.0 * rows * (double)N, 2.0 * rows * es, rows * N * es, st,
               [&](const ProfDev* pd) {
                 return launch_cov_stencil(prec, g, Z, ldz, N, V, ldv, vcols, B, Bdev, T, ldt, rows_per_wave, st, pd,
                                           zc);
               });
}

hipError_t cov_bf16_timed(const Grid& g, const float* Z, int64_t ldz, int64_t N, const __hip_bfloat16* V,
                          int64_t ldk, int64_t vcols, int64_t B, const int32_t* Bdev, float* T, int64_t ldt, int tile,
                          hipStream_t st, int32_t* zc) {
  if (!g_prof.on) return launch_cov_bf16(g, Z, ldz, N, V, ldk, vcols, B, Bdev, T, ldt, tile, st, nullptr, zc);
  const double rows = (double)g.nz * g.nx;
  // BF16 input column, FP32 output column; Z is read in FP32
  return timed(INFOESRF_PROF_OP_BF16, 2.0 * (double)N * grid_nnz(g) + 3.0 * rows * (double)N, rows * (2.0 + 4.0),
               rows * N * 4.0, st, [&](const ProfDev* pd) {
                 return launch_cov_bf16(g, Z, ldz, N, V, ldk, vcols, B, Bdev, T, ldt, tile, st, pd, zc);
               });
}

hipError_t pcg_fused_timed(Prec prec, const PCGState& s, const LMP& lmp, int mode, int obs_domain, int plain,
                           const void* T, int64_t ldt, const int32_t* act, const int32_t* nact, int32_t* act_out,
                           int32_t* nact_out, int64_t Bmax, void* V, int64_t ldv, const int32_t* h_ptr,
                           const int32_t* h_idx, const double* h_w, const double* r_var, int64_t n_state,
                           hipStream_t st) {
  if (!g_prof.on)
    return launch_pcg_fused(prec, s, lmp, mode, obs_domain, plain, T, ldt, act, nact, act_out, nact_out, Bmax, V,
                            ldv, h_ptr, h_idx, h_w, r_var, n_state, st);
  // per live system: read r, p, x and the apply output, write x, r, p and the next apply input;
  // per launch: Phi and S Phi once.  Flops: (12 + 8p) per row.
  const double m = (double)s.m, P = (double)lmp.p;
  const double t_in = prec == Prec::F64 ? 8.0 : 4.0;
  const double v_out = prec == Prec::F64 ? 8.0 : (prec == Prec::F32 ? 4.0 : 2.0);
  const double per_vec = m * (3 * 8.0 + t_in + 3 * 8.0 + (obs_domain ? v_out : 0.0));
  return timed(INFOESRF_PROF_PCG, m * (12.0 + 8.0 * P), per_vec, 2.0 * m * P * 8.0, st, [&](const ProfDev* pd) {
    PCGState sp = s;
    sp.prof = pd ? *pd : ProfDev{};
    return launch_pcg_fused(prec, sp, lmp, mode, obs_domain, plain, T, ldt, act, nact, act_out, nact_out, Bmax, V,
                            ldv, h_ptr, h_idx, h_w, r_var, n_state, st);
  });
}

hipError_t pcg_tail_timed(const PCGState& s, const LMP& lmp, const TailApply& ap, const int32_t* act,
                          const int32_t* nact, int32_t* qctr, int64_t grid, const double* r0, double* uacc,
                          const TailCheck& chk, hipStream_t st) {
  if (!g_prof.on) return launch_pcg_tail(s, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
  // per system-iteration: the apply and the PCG step; per system: a start reads its residual and
  // reads and writes its solution, a continuation reads and writes x, r, p, and the residual check
  // reads b and writes the true residual; per launch from HBM: the band (or S) in the iterations'
  // precision and in FP64 for the check (one array when both are FP64), and the Ritz bases
  const double m = (double)s.m, P = (double)lmp.p;
  const double apply = ap.kind == 1 ? 2.0 * m * m : 2.0 * grid_nnz(ap.g);
  const double entries = ap.kind == 1 ? m * m : m * (2 * ap.g.bz + 1) * (2 * ap.g.bx + 1);
  const double matrix = entries * (ap.low ? 8.0 + 4.0 : 8.0);
  const double per_system = ((r0 ? 3.0 : 6.0) + (chk.b ? 2.0 : 0.0)) * 8.0 * m;
  return timed(INFOESRF_PROF_TAIL, apply + m * (12.0 + 8.0 * P), per_system,
               matrix + 2.0 * 8.0 * m * P, st,
               [&](const ProfDev* pd) {
                 PCGState sp = s;
                 sp.prof = pd ? *pd : ProfDev{};
                 return launch_pcg_tail(sp, lmp, ap, act, nact, qctr, grid, r0, uacc, chk, st);
               });
}

hipError_t cov_band_timed(Prec prec, const Grid& g, const void* band, int64_t ldb, const void* V, int64_t ldv,
                          int64_t vcols, int64_t B, const int32_t* Bdev, void* T, int64_t ldt, hipStream_t st,
                          int32_t* zc) {
  if (!g_prof.on) return launch_band_apply(prec, g, band, ldb, V, ldv, vcols, B, Bdev, T, ldt, st, nullptr, zc);
  const double rows = (double)g.nz * g.nx;
  const double es = (double)elem_size(prec);
  const double planes = (double)(2 * g.bz + 1) * (2 * g.bx + 1);
  const int slot = prec == Prec::F64 ? INFOESRF_PROF_BAND_FP64 : INFOESRF_PROF_BAND_FP32;
  return timed(slot, 2.0 * grid_nnz(g), 2.0 * rows * es, planes * rows * es, st, [&](const ProfDev* pd) {
    return launch_band_apply(prec, g, band, ldb, V, ldv, vcols, B, Bdev, T, ldt, st, pd, zc);
  });
}

}  // namespace infoesrf

using namespace infoesrf;

extern "C" int infoesrf_profile_enable(int on) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_prof_mu);
  if (on) {
    if (g_prof.ev.empty()) {
      g_prof.ev.resize(2 * kPairs);
      g_prof.ev_slot.resize(kPairs);
      for (auto& e : g_prof.ev) IE_HIP(hipEventCreate(&e));
      IE_HIP(hipMalloc(&g_prof.dvec, kSlots * sizeof(unsigned long long)));
      IE_HIP(hipMalloc(&g_prof.dflops, kSlots * sizeof(double)));
      IE_HIP(hipMalloc(&g_prof.dbytes, kSlots * sizeof(double)));
    }
    IE_HIP(hipDeviceSynchronize());
    IE_HIP(hipMemset(g_prof.dvec, 0, kSlots * sizeof(unsigned long long)));
    IE_HIP(hipMemset(g_prof.dflops, 0, kSlots * sizeof(double)));
    IE_HIP(hipMemset(g_prof.dbytes, 0, kSlots * sizeof(double)));
    for (int i = 0; i < kSlots; ++i) {
      g_prof.ms[i] = 0.0;
      g_prof.launches[i] = 0;
      g_prof.host_bytes[i] = 0.0;
    }
    g_prof.used = 0;
    g_prof.mask = ~0u;
  }
  g_prof.on = on != 0;
  return INFOESRF_OK;
}

extern "C" int infoesrf_profile_select(uint32_t mask) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_prof_mu);
  g_prof.mask = mask;
  return INFOESRF_OK;
}

extern "C" int infoesrf_profile_read(double ms[7], int64_t launches[7], int64_t vectors[7], double flops[7],
                                     double bytes[7]) {
  clear_error();
  IE_CHECK(ms && launches && vectors && flops && bytes, INFOESRF_ERR_INVALID_ARG, "outputs must be non-NULL");
  std::lock_guard<std::mutex> lock(g_prof_mu);
  if (!g_prof.dvec) {
    for (int i = 0; i < kSlots; ++i) {
      ms[i] = 0.0;
      launches[i] = 0;
      vectors[i] = 0;
      flops[i] = 0.0;
      bytes[i] = 0.0;
    }
    return INFOESRF_OK;
  }
  IE_HIP(hipDeviceSynchronize());
  IE_HIP(drain());
  unsigned long long v[kSlots];
  double f[kSlots], b[kSlots];
  IE_HIP(hipMemcpy(v, g_prof.dvec, sizeof(v), hipMemcpyDeviceToHost));
  IE_HIP(hipMemcpy(f, g_prof.dflops, sizeof(f), hipMemcpyDeviceToHost));
  IE_HIP(hipMemcpy(b, g_prof.dbytes, sizeof(b), hipMemcpyDeviceToHost));
  for (int i = 0; i < kSlots; ++i) {
    ms[i] = g_prof.ms[i];
    launches[i] = g_prof.launches[i];
    vectors[i] = (int64_t)v[i];
    flops[i] = f[i];
    bytes[i] = b[i] + g_prof.host_bytes[i];
  }
  return INFOESRF_OK;
}
