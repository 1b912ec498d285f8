// Per-kernel-class launch timing for roofline reporting.
//
// While a session is active for one kernel class, every launch of that class
// is bracketed by a pair of HIP events recorded on the launch stream, and the
// launch's algorithmic bytes and FLOP (computed from its shape by the
// launcher) are summed.  One session per process; not thread-safe.
#include "qtt_internal.hpp"

#include <vector>

namespace qtt {
namespace prof {

namespace {
struct State {
  int cls = -1;
  int cap = 0;
  int used = 0;
  bool open = false;
  std::vector<hipEvent_t> ev;
  double bytes = 0.0, flops = 0.0;
};
State& state() {
  static State s;
  return s;
}
}  // namespace

bool active(int cls) {
  State& s = state();
  return s.cls == cls && s.used < s.cap;
}

void begin(hipStream_t st, int cls, double bytes, double flops) {
  State& s = state();
  if (s.cls != cls || s.used >= s.cap || s.open) return;
  if (hipEventRecord(s.ev[2 * s.used], st) != hipSuccess) return;
  s.open = true;
  s.bytes += bytes;
  s.flops += flops;
}

void end(hipStream_t st) {
  State& s = state();
  if (!s.open) return;
  (void)hipEventRecord(s.ev[2 * s.used + 1], st);
  s.open = false;
  ++s.used;
}

hipError_t start(int cls, int max_launches) {
  State& s = state();
  for (hipEvent_t e : s.ev) (void)hipEventDestroy(e);
  s.ev.clear();
  s.cls = -1;
  s.used = 0;
  s.open = false;
  s.bytes = s.flops = 0.0;
  s.ev.resize(2 * (size_t)max_launches);
  for (auto& e : s.ev) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
  }
  s.cap = max_launches;
  s.cls = cls;
  return hipSuccess;
}

hipError_t stop(long* launches, double* total_ms, double* bytes, double* flops) {
  State& s = state();
  double tot = 0.0;
  if (s.used > 0) {
    hipError_t r = hipEventSynchronize(s.ev[2 * s.used - 1]);
    if (r != hipSuccess) return r;
  }
  for (int i = 0; i < s.used; ++i) {
    float ms = 0.f;
    hipError_t r = hipEventElapsedTime(&ms, s.ev[2 * i], s.ev[2 * i + 1]);
    if (r != hipSuccess) return r;
    tot += ms;
  }
  *launches = s.used;
  *total_ms = tot;
  *bytes = s.bytes;
  *flops = s.flops;
  for (hipEvent_t e : s.ev) (void)hipEventDestroy(e);
  s.ev.clear();
  s.cls = -1;
  s.cap = s.used = 0;
  return hipSuccess;
}

}  // namespace prof
}  // namespace qtt
