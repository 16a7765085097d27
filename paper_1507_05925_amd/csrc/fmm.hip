// 2D fast multipole far field (placeholder until the tree code lands).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace bie {

struct FmmPlan {};

int fmm_far_field(bie_geom *, int, int, int, const double *, double *, hipStream_t, int, int) {
  set_error("BIE_FMM is not available in this build");
  return BIE_EINVAL;
}

void fmm_destroy(FmmPlan *p) { delete p; }

int fmm_current_order() { return 0; }

}  // namespace bie
