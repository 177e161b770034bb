// Named ranges for profiler timelines (roctx; seen with rocprofv3 --marker-trace, no cost
// otherwise): setup phases, device layout, solves, autotuning, the nested start.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace asmg {

struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace asmg
