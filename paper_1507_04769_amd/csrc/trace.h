// roctx ranges around the C-ABI calls: a profiler that records markers
// (rocprofv3 --marker-trace) shows every call as a named range on the
// calling thread, beside the kernels it launched.  Without such a tool the
// calls cost a few nanoseconds.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace sgcm {

struct CallRange {
  explicit CallRange(const char* name) { roctxRangePushA(name); }
  ~CallRange() { roctxRangePop(); }
  CallRange(const CallRange&) = delete;
  CallRange& operator=(const CallRange&) = delete;
};

}  // namespace sgcm
