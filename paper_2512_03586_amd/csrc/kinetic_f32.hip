// kinetic_f32.hip -- kinetic IMEX stage kernels with float storage of f.
#include "kinetic_impl.h"

namespace esbgk {
ESBGK_INST(float)
}  // namespace esbgk
