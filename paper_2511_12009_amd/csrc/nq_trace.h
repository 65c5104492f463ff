// Named host ranges for the profiler's marker trace (rocprofv3 --marker-trace):
// the phases of a count (frontier, expansion, DFS launch, result copy), chunks
// of a chunked count, batch set-up and replay, and serving epochs.  Without a
// profiler attached the calls return at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace nqi {

class TraceRange {
public:
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace nqi
