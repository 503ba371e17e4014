// Process-wide table of measured block shapes for the covariance applies (see
// infoesrf_autotune).  Keys are the apply's grid and form; values are the fastest choice per
// batch-size bucket.  Reads and writes take a lock; the tuner sets a thread-local override while
// it times candidates.
#include <map>
#include <mutex>
#include <tuple>

#include "internal.hpp"

namespace infoesrf {

thread_local int g_force_choice = 0;

namespace {
using Key = std::tuple<int, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<Key, std::array<int, kTuneBuckets>> g_tune;
Key key_of(const TuneKey& k) { return Key{k.form, k.prec, k.nz, k.nx, k.bz, k.bx, k.N}; }
}  // namespace

int tune_bucket(int64_t B) { return B >= 256 ? 0 : (B >= 64 ? 1 : 2); }

int tuned_choice(const TuneKey& k, int64_t B) {
  if (g_force_choice) return g_force_choice;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(key_of(k));
  if (it == g_tune.end()) return 0;
  return it->second[tune_bucket(B)];
}

void set_tuned(const TuneKey& k, int bucket, int choice) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto& row = g_tune[key_of(k)];
  row[bucket] = choice;
}

void tune_reset() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
}

}  // namespace infoesrf
