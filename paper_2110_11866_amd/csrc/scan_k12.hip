// Scan kernels with 12 Fourier terms (see scan_kernel.h).
#include "scan_kernel.h"

namespace mk {
KernelFn select_scan_k12(int R, int var, int wide, int gauss, int mom) {
  if (R == 8) return pick_scan<12, 8>(var, wide, gauss, mom);
  if (R == 16) return pick_scan<12, 16>(var, wide, gauss, mom);
  return nullptr;
}
}  // namespace mk
