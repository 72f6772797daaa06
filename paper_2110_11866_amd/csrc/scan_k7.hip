// Scan kernels with 7 Fourier terms (see scan_kernel.h).
#include "scan_kernel.h"

namespace mk {
KernelFn select_scan_k7(int R, int var, int wide, int gauss, int mom) {
  if (R == 8) return pick_scan<7, 8>(var, wide, gauss, mom);
  if (R == 16) return pick_scan<7, 16>(var, wide, gauss, mom);
  return nullptr;
}
}  // namespace mk
