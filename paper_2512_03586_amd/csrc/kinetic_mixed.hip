// kinetic_mixed.hip -- kinetic IMEX stage kernels of the mixed storage form:
// the state f^n (and f^{n+1}) in float, the stage arrays f^(2), f^(3) in BF16.
#include "kinetic_impl.h"

namespace esbgk {
ESBGK_INST_STAGE(float, bf16_t)
}  // namespace esbgk
