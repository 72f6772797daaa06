// Forward scan kernels with 10 Fourier terms (see scan_fwd_kernel.h).
#include "scan_fwd_kernel.h"

namespace mk {
KernelFn select_fwd_k10(int R, int wide, int kind) {
  if (R == 8) return pick_fwd<10, 8>(wide, kind);
  if (R == 16) return pick_fwd<10, 16>(wide, kind);
  return nullptr;
}
}  // namespace mk
