// dirac_trace.h -- named host ranges around the library's entry points, for
// rocprofv3's marker trace (--marker-trace): each call appears as a range
// ("dl_step", "dl_observables", ...) on the host timeline, next to the
// kernels it enqueued.  Without a tool attached a range costs two calls into
// the roctx library.  Internal to libdirac.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace dirac {

class TraceRange {
 public:
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace dirac
