// Status codes, per-thread error text and device queries.
#include <cstring>
#include <mutex>

#include "common.hpp"

namespace hg {

static thread_local char g_last_error[512] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
}

void clear_error() { g_last_error[0] = '\0'; }

int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

}  // namespace hg

extern "C" const char *hg_status_str(int status) {
  switch (status) {
    case HG_OK: return "HG_OK";
    case HG_EINVAL: return "HG_EINVAL: invalid argument";
    case HG_EHIP: return "HG_EHIP: HIP runtime error";
    case HG_EWORKSPACE: return "HG_EWORKSPACE: workspace missing or too small";
    case HG_EUNSUPPORTED: return "HG_EUNSUPPORTED: not supported";
    default: return "unknown status";
  }
}

extern "C" const char *hg_last_error(void) { return hg::g_last_error; }

extern "C" int hg_version(void) { return 10000; }
