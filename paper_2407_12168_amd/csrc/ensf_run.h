// Internal: workspace-level entry of one analysis and the two small kernels it needs to run
// without host-to-device copies or memsets (so the caller may capture it in a graph).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/ensf.h"

namespace ensf {

// Zeroes `bytes` bytes at the device address p (a kernel, not hipMemsetAsync).
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// Copies `bytes` bytes of host memory src to the device address dst by passing them as
// kernel arguments (the host buffer may be reused as soon as this returns).
hipError_t launch_put_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);

// Bytes one analysis of problem p with options o needs in run_in_workspace's buffer.
size_t workspace_bytes(const ensf_options& o, const ensf_problem& p);

// One analysis of problem p (ensf_analysis semantics) with every device buffer carved out of
// ws (ws_bytes, 256-byte aligned), the pseudo-time loop launched eagerly on s, and the
// device counters (non-finite particle values, invalid observations) added to counters[0..1].
// Allocates no device or pinned memory.  ENSF_ESCRATCH when ws_bytes is too small.
ensf_status run_in_workspace(const ensf_options& o, const ensf_problem& p, char* ws,
                             size_t ws_bytes, unsigned long long* counters, hipStream_t s);

}  // namespace ensf
