// Host-side parts of the C ABI that launch nothing: version, status names,
// word counts and the per-device architecture check.
#include <hip/hip_runtime.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bs_common.h"

namespace bs {

// ---- opt-in kernel timing with HIP events ------------------------------------
namespace {
struct Pending {
  std::string name;
  hipEvent_t start, stop;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<double, int64_t>> g_totals;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

ScopedTiming::ScopedTiming(const char* name, hipStream_t s) : name_(name), s_(s) {
  std::lock_guard<std::mutex> lock(g_tmu);
  if (!g_timing || !name_) return;  // a null name: never timed (creates no events)
  // launches recorded into a graph are timed only as a whole, by the caller
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  start_ = take_event();
  stop_ = take_event();
  if (start_ && stop_) (void)hipEventRecord(start_, s_);
}

ScopedTiming::~ScopedTiming() {
  std::lock_guard<std::mutex> lock(g_tmu);
  if (!start_ || !stop_) return;
  (void)hipEventRecord(stop_, s_);
  g_pending.push_back(Pending{name_, start_, stop_});
}

void device_limits(int* lds_max, int* n_cu) {
  static std::mutex mu;
  static int cache[64][2];
  static bool have[64] = {false};
  int dev = 0;
  *lds_max = 0;
  *n_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lock(mu);
  if (!have[dev]) {
    int l = 0, c = 0;
    if (hipDeviceGetAttribute(&l, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      l = 0;
      c = 0;
    }
    cache[dev][0] = l;
    cache[dev][1] = c;
    have[dev] = true;
  }
  *lds_max = cache[dev][0];
  *n_cu = cache[dev][1];
}

bs_status check_device() {
  static std::mutex mu;
  static int known[64] = {0};  // 0 unknown, 1 gfx950, 2 other
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BS_ERR_DEVICE;
  if (dev < 0 || dev >= 64) return BS_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(mu);
  if (known[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return BS_ERR_DEVICE;
    known[dev] = strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
  }
  return known[dev] == 1 ? BS_OK : BS_ERR_DEVICE;
}

}  // namespace bs

extern "C" int bs_version(void) { return 10000; }

extern "C" const char* bs_status_string(int status) {
  switch (status) {
    case BS_OK:
      return "ok";
    case BS_ERR_NULL:
      return "a required pointer is NULL";
    case BS_ERR_ARG:
      return "a size or parameter is out of range";
    case BS_ERR_WORKSPACE:
      return "workspace missing, misaligned or too small";
    case BS_ERR_HIP:
      return "the HIP runtime rejected a launch";
    case BS_ERR_DEVICE:
      return "the current device is not a gfx950";
    case BS_ERR_SCRATCH:
      return "the call needs more than the fixed no-allocation scratch (BS_NOALLOC_SCRATCH_BYTES)";
    default:
      return "unknown status";
  }
}

extern "C" int32_t bs_words(int32_t N) { return bs::valid_width(N) ? N / 64 : 0; }

extern "C" int bs_timing_enable(int on) {
  std::lock_guard<std::mutex> lock(bs::g_tmu);
  bs::g_timing = on != 0;
  return 0;
}

extern "C" int bs_timing_collect(void) {
  std::lock_guard<std::mutex> lock(bs::g_tmu);
  int bad = 0;
  for (auto& p : bs::g_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      auto& t = bs::g_totals[p.name];
      t.first += ms;
      t.second += 1;
    } else {
      ++bad;
    }
    bs::g_pool.push_back(p.start);
    bs::g_pool.push_back(p.stop);
  }
  bs::g_pending.clear();
  return bad;
}

extern "C" void bs_timing_reset(void) {
  std::lock_guard<std::mutex> lock(bs::g_tmu);
  bs::g_totals.clear();
}

extern "C" int bs_timing_get(const char* name, double* total_ms, int64_t* count) {
  std::lock_guard<std::mutex> lock(bs::g_tmu);
  auto it = bs::g_totals.find(name ? name : "");
  if (it == bs::g_totals.end()) {
    if (total_ms) *total_ms = 0.0;
    if (count) *count = 0;
    return 0;
  }
  if (total_ms) *total_ms = it->second.first;
  if (count) *count = it->second.second;
  return 1;
}
