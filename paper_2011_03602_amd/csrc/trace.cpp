// Named host ranges (ROCTx) around the offloaded nests, the planned
// transfers, graph launches, batched runs and tuner measurements, so that a
// marker trace (rocprofv3 --marker-trace) shows which phase of the offloaded
// program issued which kernels and copies. A range covers the host-side issue
// of its work, not the GPU time (the kernel trace gives that). With no tool
// attached each call returns at once.
#include <rocprofiler-sdk-roctx/roctx.h>

#include "ofl_internal.hpp"

namespace ofl {

void trace_push(const char *name) { roctxRangePush(name); }

void trace_pop() { roctxRangePop(); }

}  // namespace ofl
