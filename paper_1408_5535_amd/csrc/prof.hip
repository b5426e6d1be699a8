// Event-pair timing of selected kernels, enabled by phsvds_profile().
// Pairs are recorded on the launching stream; elapsed times are harvested
// when the pool fills and when results are read.
#include "prof.hpp"

#include <mutex>
#include <vector>

#include "../../include/phsvds.h"
#include "common.hpp"

namespace phs {
namespace {

struct Rec {
  hipEvent_t a, b;
  int kind, count;
  double bytes;
};

struct Prof {
  std::mutex mu;
  bool on = false;
  int mask = 0;   // kinds recorded (bit k = kind k)
  int every = 1;  // time one pair of consecutive operations in `every`
  int64_t calls[kProfCount] = {};
  std::vector<hipEvent_t> pool;
  std::vector<Rec> live;
  hipEvent_t pending = nullptr;
  int pending_kind = -1;
  int group_kind = -1, group_count = 0;  // an open group (prof_group_begin)
  int64_t n[kProfCount] = {};
  double sec[kProfCount] = {}, bytes[kProfCount] = {};
} g;

hipEvent_t get_event() {
  if (!g.pool.empty()) {
    hipEvent_t e = g.pool.back();
    g.pool.pop_back();
    return e;
  }
  // Timing-only events: without the system-scope fence the interval does
  // not include a cache write-back after the kernel.
  hipEvent_t e;
  PHS_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  return e;
}

void harvest() {
  for (Rec &r : g.live) {
    PHS_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    PHS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    g.n[r.kind] += r.count;
    g.sec[r.kind] += ms * 1e-3;
    g.bytes[r.kind] += r.bytes;
    g.pool.push_back(r.a);
    g.pool.push_back(r.b);
  }
  g.live.clear();
}

}  // namespace

bool prof_on() { return g.on; }

void prof_begin(int kind, hipStream_t s) {
  if (!g.on || !((g.mask >> kind) & 1) || g.group_kind == kind) return;
  std::lock_guard<std::mutex> lk(g.mu);
  // sampling by pairs keeps A X and the A^T Y that follows it together
  const int64_t c = g.calls[kind]++;
  if ((c / 2) % g.every != 0) {
    g.pending = nullptr;
    return;
  }
  g.pending = get_event();
  g.pending_kind = kind;
  PHS_HIP(hipEventRecord(g.pending, s));
}

void prof_end(int kind, hipStream_t s, double bytes) {
  if (!g.on || !((g.mask >> kind) & 1) || g.group_kind == kind) return;
  std::lock_guard<std::mutex> lk(g.mu);
  if (!g.pending || g.pending_kind != kind) return;
  hipEvent_t e = get_event();
  PHS_HIP(hipEventRecord(e, s));
  g.live.push_back({g.pending, e, kind, 1, bytes});
  g.pending = nullptr;
  if (g.live.size() >= 4096) harvest();
}

void prof_group_begin(int kind, hipStream_t s, int count) {
  if (!g.on || !((g.mask >> kind) & 1)) return;
  std::lock_guard<std::mutex> lk(g.mu);
  g.group_kind = kind;
  g.group_count = count;
  const int64_t c = g.calls[kind];
  g.calls[kind] += count;
  if ((c / 2) % g.every != 0) {
    g.pending = nullptr;
    return;
  }
  g.pending = get_event();
  g.pending_kind = kind;
  PHS_HIP(hipEventRecord(g.pending, s));
}

void prof_group_end(int kind, hipStream_t s, double bytes) {
  if (!g.on || !((g.mask >> kind) & 1)) return;
  std::lock_guard<std::mutex> lk(g.mu);
  const int count = g.group_count;
  g.group_kind = -1;
  g.group_count = 0;
  if (!g.pending || g.pending_kind != kind) return;
  hipEvent_t e = get_event();
  PHS_HIP(hipEventRecord(e, s));
  g.live.push_back({g.pending, e, kind, count, bytes});
  g.pending = nullptr;
  if (g.live.size() >= 4096) harvest();
}

}  // namespace phs

extern "C" {

int phsvds_profile(int enable) {
  try {
    std::lock_guard<std::mutex> lk(phs::g.mu);
    phs::harvest();
    if (enable) {
      for (int k = 0; k < phs::kProfCount; ++k) {
        phs::g.n[k] = 0;
        phs::g.calls[k] = 0;
        phs::g.sec[k] = phs::g.bytes[k] = 0.0;
      }
      phs::g.every = 1;
    }
    phs::g.group_kind = -1;
    phs::g.group_count = 0;
    phs::g.on = enable != 0;
    phs::g.mask = enable == 1 ? (1 << phs::kProfCount) - 1 : (enable >> 1);
    return PHSVDS_OK;
  } catch (const phs::Error &e) {
    return e.code;
  }
}

int phsvds_profile_sample(int every) {
  if (every < 1) return PHSVDS_EINVAL;
  std::lock_guard<std::mutex> lk(phs::g.mu);
  phs::g.every = every;
  for (int k = 0; k < phs::kProfCount; ++k) phs::g.calls[k] = 0;
  return PHSVDS_OK;
}

int phsvds_profile_read(int kind, int64_t *launches, double *seconds, double *bytes) {
  if (kind < 0 || kind >= phs::kProfCount || !launches || !seconds || !bytes)
    return PHSVDS_EINVAL;
  try {
    std::lock_guard<std::mutex> lk(phs::g.mu);
    phs::harvest();
    *launches = phs::g.n[kind];
    *seconds = phs::g.sec[kind];
    *bytes = phs::g.bytes[kind];
    return PHSVDS_OK;
  } catch (const phs::Error &e) {
    return e.code;
  }
}

}  // extern "C"
