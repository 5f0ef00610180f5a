// zmc_trace.hpp -- named host-side ranges for the ROCTx marker timeline.
//
// `rocprofv3 --marker-trace` records each range with its start and end time
// on the calling thread, beside the kernel trace, so that the phases of an
// entry point (staging, planning, launches, a server's admissions and
// slices) can be lined up with the kernels they enqueue.  Without a tool
// attached a range costs two calls into the ROCTx library that return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace zmc {

// A range from construction to the end of the enclosing scope.  `name` must
// be a string that outlives the call (a literal).
class TraceRange {
 public:
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace zmc
