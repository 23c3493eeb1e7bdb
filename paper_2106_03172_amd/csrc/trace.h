// Named host ranges for timeline profilers (roctx).  A range covers the host
// call that enqueues a phase (matrix build, epoch call, anchor pass, objective,
// projector call, serving tick, checkpoint); the kernels it enqueued appear in
// the same profiler's kernel trace.  With no profiler attached a push or pop is
// a call through a null hook.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace svr {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

// range names of the epoch calls, by algorithm code (svr_algo)
inline const char *epoch_range_name(int algo) {
    static const char *const names[] = {"svr.epoch.osem", "svr.epoch.svrem", "svr.epoch.svrg", "svr.epoch.saga",
                                        "svr.epoch.sga",  "svr.epoch.bsrem", "svr.epoch.sem",  "svr.epoch.sagaem"};
    return (algo >= 0 && algo < (int)(sizeof(names) / sizeof(names[0]))) ? names[algo] : "svr.epoch";
}

}  // namespace svr
