// Host-side trace ranges (roctx): visible with `rocprofv3 --marker-trace`,
// a no-op call when no profiler is attached.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace igm {

// Marks the lifetime of the object as a named range on the calling thread.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace igm
