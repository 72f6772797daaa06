// Host-only stand-ins for the library's device-side launchers, so that the host sources
// (api.cpp, plan.cpp) can be built with the host sanitizers by a plain C++ compiler and run
// without a GPU. No plan made here has a device table, so the entry points stop before any
// launch; every stand-in reports that no device is present.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "boundary.h"
#include "image2d.h"
#include "multiply.h"
#include "noalloc.h"

namespace mk {

hipError_t launch_scan(const ScanLaunch&, int, int, hipStream_t) { return hipErrorNoDevice; }
int scan_occupancy(int, int, int, int, int, int, int) { return 0; }
hipError_t launch_pg_finalize(const ScanLaunch&, int, double*, double*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_sum_scales(const float*, float*, const Row*, int, int, int64_t, hipStream_t) { return hipErrorNoDevice; }
int direct_conv_slabs(int64_t, int64_t, int) { return 1; }
hipError_t launch_direct_conv(const void*, int, int64_t, const float2*, int64_t, int, float2*, float2*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_scan_forward(const ScanLaunch&, hipStream_t) { return hipErrorNoDevice; }
int scan_forward_occupancy(int, int, int, int) { return 0; }
hipError_t launch_zero_fill(void*, size_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_mm_demodulate(const void*, int, float*, int64_t, double, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_mm_remodulate(const float*, float2*, int64_t, double, double, double, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_mm_remodulate_t(const float2*, float*, int64_t, double, double, double, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_mm_demodulate_t(const float*, float*, int64_t, double, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_transpose(const float*, float*, int64_t, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_transpose_c2p(const float2*, float*, int64_t, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_transpose_p2c(const float*, float2*, int64_t, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_tree(const void*, int, int64_t, int64_t, int, int, const TreeCoef&, int, float2*, void*, hipStream_t) {
  return hipErrorNoDevice;
}
hipError_t launch_edge_extend(const void*, int, int64_t, int64_t, float*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_pad_center(const void*, int, int64_t, int64_t, void*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_edge_fold(const float*, int64_t, int64_t, float*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_reverse(const float*, float*, int64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t scratch_setup(int) { return hipErrorNoDevice; }
void* scratch_ptr(int) { return nullptr; }

}  // namespace mk
