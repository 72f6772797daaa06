// One (K, R) set of scan kernel instantiations (see scan_kernel.h). The build compiles this
// file once per pair, with -DMK_K=<terms> -DMK_R=<samples per thread>, so the pairs build in
// parallel.
#include "scan_kernel.h"

#if !defined(MK_K) || !defined(MK_R)
#error "compile with -DMK_K=<1..12> -DMK_R=<4|8|16|32>"
#endif

#define MK_SELECT_NAME_(k, r) select_scan_k##k##_r##r
#define MK_SELECT_NAME(k, r) MK_SELECT_NAME_(k, r)

namespace mk {
KernelFn MK_SELECT_NAME(MK_K, MK_R)(int var, int acc, int kind, int mom, int dt) {
#if defined(MK_STUB)
  // development builds of a subset of (K, R): this pair has no kernels
  (void)var; (void)acc; (void)kind; (void)mom; (void)dt;
  return nullptr;
#else
  return pick_scan<MK_K, MK_R>(var, acc, kind, mom, dt);
#endif
}
}  // namespace mk
