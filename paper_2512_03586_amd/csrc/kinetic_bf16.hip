// kinetic_bf16.hip -- kinetic IMEX stage kernels with bf16_t storage of f.
#include "kinetic_impl.h"

namespace esbgk {
ESBGK_INST(bf16_t)
}  // namespace esbgk
