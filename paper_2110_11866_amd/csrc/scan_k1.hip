// Scan kernels with 1 Fourier term (see scan_kernel.h).
#include "scan_kernel.h"

namespace mk {
KernelFn select_scan_k1(int R, int var, int wide, int gauss, int mom, int dt) {
  if (R == 16) return pick_scan<1, 16>(var, wide, gauss, mom, dt);
  if (R == 32) return pick_scan<1, 32>(var, wide, gauss, mom, dt);
  return nullptr;
}
}  // namespace mk
