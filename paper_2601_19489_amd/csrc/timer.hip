// Kernel tuning state, and the launch timer: when enabled for a kernel name, every launch of that kernel
// is bracketed by two HIP events recorded on the kernel's own stream; the
// accumulated device time is read back (and reset) on request.
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace gs {

namespace {
std::mutex g_mu;
std::string g_target;
std::atomic<bool> g_on{false};
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::vector<Rec> g_events;
}  // namespace

thread_local const char* t_name = nullptr;

void timer_begin(const char* name, hipStream_t st, hipEvent_t* a, hipEvent_t* b) {
  *a = *b = nullptr;
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || (g_target != "*" && g_target != name)) return;
  t_name = name;
  if (hipEventCreate(a) != hipSuccess || hipEventCreate(b) != hipSuccess) {
    *a = *b = nullptr;
    return;
  }
  hipEventRecord(*a, st);
}

void timer_end(hipStream_t st, hipEvent_t a, hipEvent_t b) {
  if (!a) return;
  hipEventRecord(b, st);
  std::lock_guard<std::mutex> lk(g_mu);
  g_events.push_back(Rec{t_name ? t_name : "", a, b});
}

// one set of knobs per host thread: launches from one thread never see another
// thread's settings
thread_local gs_tuning g_tuning = {1, 4, 12, 0, 0, 0, {0, 0}};
const gs_tuning& tuning() { return g_tuning; }

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_set_tuning(const gs_tuning* t) {
  if (!t) return GS_EINVAL;
  if (t->fwd_px != 1 && t->fwd_px != 2 && t->fwd_px != 4) return GS_EINVAL;
  if (t->bwd_px != 1 && t->bwd_px != 2 && t->bwd_px != 4) return GS_EINVAL;
  if (t->persist_wgs < 1 || t->persist_wgs > 32) return GS_EINVAL;
  if (t->seq_walk != 0 && t->seq_walk != 1) return GS_EINVAL;
  if (t->fwd_batch != 0 && t->fwd_batch != 64 && t->fwd_batch != 128 && t->fwd_batch != 256)
    return GS_EINVAL;
  if (t->bwd_batch != 0 && t->bwd_batch != 32 && t->bwd_batch != 64 && t->bwd_batch != 128)
    return GS_EINVAL;
  g_tuning = *t;
  return GS_OK;
}

extern "C" gs_status gs_get_tuning(gs_tuning* t) {
  if (!t) return GS_EINVAL;
  *t = g_tuning;
  return GS_OK;
}

extern "C" gs_status gs_timer_enable(const char* kernel_name) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = kernel_name != nullptr;
  g_target = kernel_name ? kernel_name : "";
  return GS_OK;
}

extern "C" gs_status gs_timer_read(const char* kernel_name, double* total_ms,
                                   int64_t* launches) {
  if (!total_ms || !launches) return GS_EINVAL;
  std::vector<Rec> ev;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    std::vector<Rec> keep;
    for (auto& r : g_events) {
      if (!kernel_name || r.name == kernel_name)
        ev.push_back(r);
      else
        keep.push_back(r);
    }
    g_events.swap(keep);
  }
  double tot = 0.0;
  gs_status st = GS_OK;
  for (auto& e : ev) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess)
      st = GS_EHIP;
    tot += ms;
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  *total_ms = tot;
  *launches = (int64_t)ev.size();
  return st;
}
