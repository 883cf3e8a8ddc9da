// kinetic_f64.hip -- kinetic IMEX stage kernels with double storage of f.
#include "kinetic_impl.h"

namespace esbgk {
ESBGK_INST(double)
}  // namespace esbgk
