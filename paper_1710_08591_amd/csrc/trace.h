// roctx ranges around the library's C-ABI calls and serving batches, so a
// trace (rocprofv3 --marker-trace) shows which call issued which kernels.
// Without a tool attached a range costs two calls into the roctx library.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace fftbf {

class TraceRange {
 public:
  explicit TraceRange(const char* name) { roctxRangePush(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace fftbf

#define FFTBF_TRACE(name) ::fftbf::TraceRange fftbf_trace_range_(name)
