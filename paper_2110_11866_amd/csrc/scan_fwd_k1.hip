// Forward scan kernels with 1 Fourier term (see scan_fwd_kernel.h).
#include "scan_fwd_kernel.h"

namespace mk {
KernelFn select_fwd_k1(int R, int wide, int kind) {
  if (R == 8) return pick_fwd<1, 8>(wide, kind);
  if (R == 16) return pick_fwd<1, 16>(wide, kind);
  return nullptr;
}
}  // namespace mk
