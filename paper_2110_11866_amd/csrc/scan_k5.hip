// Scan kernels with 5 Fourier terms (see scan_kernel.h).
#include "scan_kernel.h"

namespace mk {
KernelFn select_scan_k5(int R, int var, int wide, int gauss, int mom, int dt) {
  if (R == 16) return pick_scan<5, 16>(var, wide, gauss, mom, dt);
  if (R == 32) return pick_scan<5, 32>(var, wide, gauss, mom, dt);
  return nullptr;
}
}  // namespace mk
