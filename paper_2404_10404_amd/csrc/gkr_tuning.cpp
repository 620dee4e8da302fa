// Round-schedule tunables. Proofs read one consistent snapshot when they are
// queued; changing the tuning never changes proof bytes, only launch shapes.
#include <atomic>

#include "gkr_tuning.hpp"

namespace gkr {

static std::atomic<uint32_t> g_tail_log{10};
static std::atomic<uint32_t> g_max_round_blocks{2048};
static std::atomic<uint32_t> g_pairs_per_thread{1};
static std::atomic<uint32_t> g_matrix_cores{1};

Tuning current_tuning() {
  Tuning t;
  t.tail_log = g_tail_log.load(std::memory_order_relaxed);
  t.max_round_blocks = g_max_round_blocks.load(std::memory_order_relaxed);
  t.pairs_per_thread = g_pairs_per_thread.load(std::memory_order_relaxed);
  t.matrix_cores = g_matrix_cores.load(std::memory_order_relaxed);
  return t;
}

void store_tuning(const Tuning& t) {
  g_tail_log.store(t.tail_log, std::memory_order_relaxed);
  g_max_round_blocks.store(t.max_round_blocks, std::memory_order_relaxed);
  g_pairs_per_thread.store(t.pairs_per_thread, std::memory_order_relaxed);
  g_matrix_cores.store(t.matrix_cores, std::memory_order_relaxed);
}

}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_set_tuning(uint32_t tail_log, uint32_t max_round_blocks, uint32_t pairs_per_thread) {
  if (tail_log < 1 || tail_log > 20 || max_round_blocks < 1 || max_round_blocks > kMaxRoundBlocks ||
      pairs_per_thread < 1 || pairs_per_thread > 1024) {
    set_error("tuning out of range");
    return GKR_EINVAL;
  }
  Tuning t = current_tuning();
  t.tail_log = tail_log;
  t.max_round_blocks = max_round_blocks;
  t.pairs_per_thread = pairs_per_thread;
  store_tuning(t);
  return GKR_OK;
}

extern "C" int32_t gkr_set_contraction(uint32_t matrix_cores) {
  if (matrix_cores > 1) {
    set_error("contraction mode out of range");
    return GKR_EINVAL;
  }
  g_matrix_cores.store(matrix_cores, std::memory_order_relaxed);
  return GKR_OK;
}

extern "C" int32_t gkr_get_contraction(uint32_t* matrix_cores) {
  if (matrix_cores) *matrix_cores = g_matrix_cores.load(std::memory_order_relaxed);
  return GKR_OK;
}

extern "C" int32_t gkr_get_tuning(uint32_t* tail_log, uint32_t* max_round_blocks, uint32_t* pairs_per_thread) {
  const Tuning t = current_tuning();
  if (tail_log) *tail_log = t.tail_log;
  if (max_round_blocks) *max_round_blocks = t.max_round_blocks;
  if (pairs_per_thread) *pairs_per_thread = t.pairs_per_thread;
  return GKR_OK;
}
