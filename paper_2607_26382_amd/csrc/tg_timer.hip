// Per-kernel-class timing with HIP events recorded on the launch stream.
// When enabled, every launch of a timed class is bracketed by two events and
// its algorithmic byte count is recorded; durations are harvested lazily.
#include <mutex>

#include "tg_internal.h"

namespace tg {

namespace {
struct Pending {
  hipEvent_t a, b;
  int kind;
  double bytes;
};
struct Acc {
  double ms = 0, bytes = 0;
  long long n = 0;
};
struct Timer {
  unsigned mask = 0;
  std::mutex mu;
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  Acc acc[TG_KT_COUNT];
};
Timer& T() {
  static Timer t;
  return t;
}
hipEvent_t get_event(Timer& t) {
  if (!t.pool.empty()) {
    hipEvent_t e = t.pool.back();
    t.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timer_on() { return T().mask != 0; }

// While a stream is being captured into a graph no events are recorded.
static thread_local bool g_suspended = false;
void timer_suspend(bool on) { g_suspended = on; }

void* timer_begin(int kind, hipStream_t s) {
  Timer& t = T();
  if (g_suspended || !((t.mask >> kind) & 1u)) return nullptr;
  std::lock_guard<std::mutex> g(t.mu);
  hipEvent_t a = get_event(t), b = get_event(t);
  if (!a || !b) return nullptr;
  hipEventRecord(a, s);
  t.pending.push_back({a, b, kind, 0.0});
  return (void*)(t.pending.size());   // 1-based index
}

void timer_end(void* h, double bytes, hipStream_t s) {
  Timer& t = T();
  if (!h) return;
  std::lock_guard<std::mutex> g(t.mu);
  Pending& p = t.pending[(size_t)h - 1];
  p.bytes = bytes;
  hipEventRecord(p.b, s);
}

void timer_harvest() {
  Timer& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto& p : t.pending) {
    hipEventSynchronize(p.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      t.acc[p.kind].ms += ms;
      t.acc[p.kind].bytes += p.bytes;
      t.acc[p.kind].n += 1;
    }
    t.pool.push_back(p.a);
    t.pool.push_back(p.b);
  }
  t.pending.clear();
}

}  // namespace tg

using namespace tg;

static const char* kNames[TG_KT_COUNT] = {"apply_f64", "vcycle_fine_op", "vcycle_coarse_op", "transfer",
                                          "multidot", "vector_update", "scalar", "setup", "fidelity"};

extern "C" {
int tg_timer_enable(int mask) {
  Timer& t = T();
  timer_harvest();
  t.mask = (unsigned)mask;
  return TG_OK;
}
int tg_timer_reset(void) {
  timer_harvest();
  Timer& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  for (auto& a : t.acc) a = Acc();
  return TG_OK;
}
int tg_timer_read(int kind, double* total_ms, long long* launches, double* bytes) {
  if (kind < 0 || kind >= TG_KT_COUNT || !total_ms || !launches || !bytes)
    return fail(TG_EINVAL, "bad timer kind or NULL output");
  timer_harvest();
  Timer& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  *total_ms = t.acc[kind].ms;
  *launches = t.acc[kind].n;
  *bytes = t.acc[kind].bytes;
  return TG_OK;
}
const char* tg_timer_name(int kind) {
  if (kind < 0 || kind >= TG_KT_COUNT) return "";
  return kNames[kind];
}
}
