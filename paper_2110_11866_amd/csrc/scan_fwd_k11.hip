// Forward scan kernels with 11 Fourier terms (see scan_fwd_kernel.h).
#include "scan_fwd_kernel.h"

namespace mk {
KernelFn select_fwd_k11(int R, int wide, int kind) {
  if (R == 8) return pick_fwd<11, 8>(wide, kind);
  if (R == 16) return pick_fwd<11, 16>(wide, kind);
  return nullptr;
}
}  // namespace mk
