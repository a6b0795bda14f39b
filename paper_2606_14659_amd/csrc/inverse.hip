// inverse.hip -- inverse iteration with conjugate gradients (paper Sec. 7,
// Alg. 2) for all segments of a bisection level.
#include "common.h"
#include "kernels.h"

namespace rsb {

int64_t inverse_level(Level &L, CompDev &C, SolveDev &S, const InverseParams &p,
                      double *y64_out, Ctx &ctx) {
  (void)L; (void)C; (void)S; (void)p; (void)y64_out; (void)ctx;
  fail(RSB_EINVAL, "method RSB_INVERSE_CG is not available in this build");
}

}  // namespace rsb
