// Host-side plumbing shared by the libhomog translation units: error
// reporting, argument checks and launch helpers. No device arithmetic here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "homog.h"

namespace hg {

void set_error(const char *fmt, ...);
void clear_error();

// Record a message and return `status`.
inline int fail(int status, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error("%s", buf);
  return status;
}

#define HG_REQUIRE(cond, ...)                                   \
  do {                                                          \
    if (!(cond)) return ::hg::fail(HG_EINVAL, __VA_ARGS__);     \
  } while (0)

#define HG_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::hg::fail(HG_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

// Check the launch that was just issued.
inline int launched(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HG_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return HG_OK;
}

inline bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Compute units of the current device (cached per device).
int device_cus();

}  // namespace hg

// A captured sequence of launches, replayed by hg_graph_launch.
struct hg_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace hg {

// Captures what record(stream) launches into a new graph. The caller's stream
// is drained first; capture runs on a private non-blocking stream.
template <class Record>
int capture_graph(void *caller_stream, Record &&record, hg_graph **out) {
  *out = nullptr;
  HG_HIP(hipStreamSynchronize(as_stream(caller_stream)));
  hipStream_t cap;
  HG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hg_graph *g = new hg_graph{nullptr, nullptr};
  int st = HG_OK;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    st = fail(HG_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  } else {
    st = record(cap);
    e = hipStreamEndCapture(cap, &g->graph);
    if (st == HG_OK && e != hipSuccess)
      st = fail(HG_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (st == HG_OK) {
      e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
      if (e != hipSuccess) st = fail(HG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
  }
  (void)hipStreamDestroy(cap);
  if (st != HG_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st;
  }
  *out = g;
  return HG_OK;
}

}  // namespace hg
