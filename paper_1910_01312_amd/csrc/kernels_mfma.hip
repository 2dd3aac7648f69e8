// bf16 MFMA gather-SYRK for the mixed-precision Newton system (placeholder
// until the MFMA tile kernel is enabled: reports "unsupported" so the fp64
// gather-SYRK is used).
#include "dev_common.h"
#include "ssn_internal.h"

namespace ssn {
bool syrk_mfma_supported(int, int64_t) { return false; }
int64_t syrk_mfma_part_size(int64_t, int64_t) { return 1; }
void launch_syrk_mfma(const void*, int, int64_t, const int32_t*, int64_t, double*, float*, int64_t,
                      hipStream_t) {}
}  // namespace ssn
