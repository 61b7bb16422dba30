// tuning.cpp -- process-wide launch parameters (see pm_tuning in pm.h).
#include <atomic>
#include <cstdlib>

#include "pm_internal.h"

namespace pm {
namespace {

int32_t env_or(const char *name, int32_t dflt) {
  const char *e = std::getenv(name);
  if (!e) return dflt;
  const long long x = std::atoll(e);
  return x >= 1 && x <= INT32_MAX ? (int32_t)x : dflt;
}

// a percentage 0..100 (the whole value must parse)
int32_t env_pct(const char *name, int32_t dflt) {
  const char *e = std::getenv(name);
  if (!e || !*e) return dflt;
  char *end = nullptr;
  const long long x = std::strtoll(e, &end, 10);
  return *end == 0 && x >= 0 && x <= 100 ? (int32_t)x : dflt;
}

struct Store {
  std::atomic<int32_t> group_v, wave_min_count, hem_compact_min_n, reb_compact_min_n,
      contract_rows_min_nnz, contract_rows_long_pct, lp_cache, graph_bodies;
  Store() {
    const int32_t v = env_or("PM_GROUP_V", 1);
    group_v = v == 2 ? 2 : 1;
    wave_min_count = env_or("PM_WAVE_MIN_COUNT", kWaveMinCount);
    hem_compact_min_n = env_or("PM_HEM_COMPACT_MIN_N", kHemCompactMinN);
    reb_compact_min_n = env_or("PM_REB_COMPACT_MIN_N", kRebCompactMinN);
    contract_rows_min_nnz = env_or("PM_CONTRACT_ROWS_MIN_NNZ", kContractRowsMinNnz);
    contract_rows_long_pct = env_pct("PM_CONTRACT_ROWS_LONG_PCT", kContractRowsLongPct);
    const char *lc = std::getenv("PM_LP_CACHE");
    lp_cache = (lc && lc[0] == '1' && lc[1] == 0) ? 1 : 0;
    const char *gb = std::getenv("PM_GRAPH_BODIES");
    graph_bodies = (gb && gb[0] == '1' && gb[1] == 0) ? 1 : 0;
  }
};

Store &store() {
  static Store s;
  return s;
}

}  // namespace

TuningValues tuning() {
  Store &s = store();
  return TuningValues{s.group_v.load(std::memory_order_relaxed),
                      s.wave_min_count.load(std::memory_order_relaxed),
                      s.hem_compact_min_n.load(std::memory_order_relaxed),
                      s.reb_compact_min_n.load(std::memory_order_relaxed),
                      s.contract_rows_min_nnz.load(std::memory_order_relaxed),
                      s.contract_rows_long_pct.load(std::memory_order_relaxed),
                      s.lp_cache.load(std::memory_order_relaxed),
                      s.graph_bodies.load(std::memory_order_relaxed)};
}

void set_tuning(const TuningValues &t) {
  Store &s = store();
  s.group_v.store(t.group_v, std::memory_order_relaxed);
  s.wave_min_count.store(t.wave_min_count, std::memory_order_relaxed);
  s.hem_compact_min_n.store(t.hem_compact_min_n, std::memory_order_relaxed);
  s.reb_compact_min_n.store(t.reb_compact_min_n, std::memory_order_relaxed);
  s.contract_rows_min_nnz.store(t.contract_rows_min_nnz, std::memory_order_relaxed);
  s.contract_rows_long_pct.store(t.contract_rows_long_pct, std::memory_order_relaxed);
  s.lp_cache.store(t.lp_cache, std::memory_order_relaxed);
  s.graph_bodies.store(t.graph_bodies, std::memory_order_relaxed);
}

}  // namespace pm

using namespace pm;

extern "C" {

int pm_get_tuning(pm_tuning *out) {
  if (!out) return PM_EINVAL;
  const TuningValues t = tuning();
  out->group_v = t.group_v;
  out->wave_min_count = t.wave_min_count;
  out->hem_compact_min_n = t.hem_compact_min_n;
  out->reb_compact_min_n = t.reb_compact_min_n;
  out->contract_rows_min_nnz = t.contract_rows_min_nnz;
  out->contract_rows_long_pct = t.contract_rows_long_pct;
  out->lp_cache = t.lp_cache;
  out->graph_bodies = t.graph_bodies;
  return PM_OK;
}

int pm_set_tuning(const pm_tuning *t) {
  if (!t) return PM_EINVAL;
  if ((t->group_v != 1 && t->group_v != 2) || t->wave_min_count < 1 ||
      t->hem_compact_min_n < 1 || t->reb_compact_min_n < 1 || t->contract_rows_min_nnz < 1 ||
      t->contract_rows_long_pct < 0 || t->contract_rows_long_pct > 100 ||
      (t->lp_cache != 0 && t->lp_cache != 1) ||
      (t->graph_bodies != 0 && t->graph_bodies != 1))
    return PM_EINVAL;
  set_tuning(TuningValues{t->group_v, t->wave_min_count, t->hem_compact_min_n,
                          t->reb_compact_min_n, t->contract_rows_min_nnz,
                          t->contract_rows_long_pct, t->lp_cache, t->graph_bodies});
  return PM_OK;
}

}  // extern "C"
