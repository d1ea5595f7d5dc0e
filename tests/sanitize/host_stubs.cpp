// Stand-ins for the device side of libsta, so that the host code (sta_graph.cpp: validation,
// levelization, tiling and the fusion plan) can be built alone with the address and
// undefined-behaviour sanitizers and driven on the CPU.  The HIP calls here are never
// reached by the host-only entry points; they report "not supported" if they are.
#include <hip/hip_runtime.h>

#include "../../paper_2203_08395_amd/csrc/sta_internal.h"

namespace sta {
size_t scratch_bytes() { return 0; }
void drop_launches(LaunchCache& c) { c.e.clear(); }
}  // namespace sta

extern "C" {
hipError_t hipMemcpyAsync(void*, const void*, size_t, hipMemcpyKind, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipErrorNotSupported; }
hipError_t hipDeviceSynchronize(void) { return hipErrorNotSupported; }
const char* hipGetErrorString(hipError_t) { return "not supported in the host-only build"; }
}
