// Per-kernel-class timing: each launch of an instrumented class is bracketed
// by two HIP events on the launch's own stream; gkr_profile_read waits for the
// events and sums the elapsed times together with the algorithmic bytes and
// field products the host attached to each launch.
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/gkr.h"
#include "gkr_internal.hpp"
#include "gkr_profile.hpp"

namespace gkr {
namespace {

struct Record {
  int cls;
  hipEvent_t a, b;
  double bytes, mulmods;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Record> g_records;     // pending (events not yet read)
std::vector<hipEvent_t> g_pool;    // free events
struct Sum {
  uint64_t launches = 0;
  double ms = 0, bytes = 0, mulmods = 0;
};
Sum g_sum[PC_COUNT];

const char* kNames[PC_COUNT] = {"forward",        "digest",         "transcript",    "eq_tables",
                                "output_claim",   "phase1_init",    "round",         "round_sub",
                                "tail",           "tail_sub",       "phase2_tables", "copy_contract",
                                "local_contract", "small",          "convert",       "batch",
                                "g_gather",       "g_forward",      "g_claim_tables", "g_phase1_init",
                                "g_phase2_tables", "vpd_ntt",        "vpd_merkle",    "vpd_fri",
                                "vpd_other"};

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void drain_locked() {
  for (Record& r : g_records) {
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        Sum& s = g_sum[r.cls];
        s.launches++;
        s.ms += ms;
        s.bytes += r.bytes;
        s.mulmods += r.mulmods;
      }
    }
    (void)hipGetLastError();
    if (r.a) g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_records.clear();
}

}  // namespace

bool prof_on() { return g_on.load(std::memory_order_relaxed); }

int prof_begin(hipStream_t s) {
  if (!prof_on()) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  Record r{0, get_event(), get_event(), 0, 0};
  if (r.a) hipEventRecord(r.a, s);
  g_records.push_back(r);
  return (int)g_records.size() - 1;
}

void prof_end(int token, hipStream_t s, ProfClass cls, double bytes, double mulmods) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (token >= (int)g_records.size()) return;
  Record& r = g_records[token];
  r.cls = cls;
  r.bytes = bytes;
  r.mulmods = mulmods;
  if (r.b) hipEventRecord(r.b, s);
}

}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (on) {
    drain_locked();
    for (auto& s : g_sum) s = Sum();
  }
  g_on.store(on != 0);
  return GKR_OK;
}

extern "C" int32_t gkr_profile_read(gkr_profile_entry* out, uint32_t cap, uint32_t* count) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  uint32_t k = 0;
  for (int c = 0; c < PC_COUNT; ++c) {
    if (g_sum[c].launches == 0) continue;
    if (out && k < cap) {
      memset(&out[k], 0, sizeof(out[k]));
      strncpy(out[k].name, kNames[c], sizeof(out[k].name) - 1);
      out[k].launches = g_sum[c].launches;
      out[k].ms = g_sum[c].ms;
      out[k].bytes = g_sum[c].bytes;
      out[k].mulmods = g_sum[c].mulmods;
    }
    ++k;
  }
  if (count) *count = k;
  return GKR_OK;
}
