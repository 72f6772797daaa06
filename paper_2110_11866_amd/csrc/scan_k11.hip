// Scan kernels with 11 Fourier terms (see scan_kernel.h).
#include "scan_kernel.h"

namespace mk {
KernelFn select_scan_k11(int R, int var, int wide, int gauss, int mom, int dt) {
  if (R == 16) return pick_scan<11, 16>(var, wide, gauss, mom, dt);
  if (R == 32) return pick_scan<11, 32>(var, wide, gauss, mom, dt);
  return nullptr;
}
}  // namespace mk
