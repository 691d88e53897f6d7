// Host-side parts of the C ABI that launch nothing: version, status names,
// word counts and the per-device architecture check.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "bs_common.h"

namespace bs {

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
    default:
      return "unknown status";
  }
}

extern "C" int32_t bs_words(int32_t N) { return bs::valid_width(N) ? N / 64 : 0; }
