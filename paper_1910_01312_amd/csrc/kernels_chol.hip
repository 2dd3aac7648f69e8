// Blocked fp64 Cholesky for q larger than the LDS-resident kernel handles
// (placeholder: no blocked path yet, so q above the LDS limit uses PCG).
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {
int chol_blocked_max() { return 0; }
void launch_chol_solve_blocked(double*, const double*, double*, int64_t, double*, Scalars*,
                               hipStream_t) {}
}  // namespace ssn
