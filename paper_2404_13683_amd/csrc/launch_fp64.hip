// Kernel instantiations: PATH_FP64 and PATH_FP64SF, 8 (digit count unused), elements 0 and 1.
#include "launch_impl.hpp"

namespace ovfem {

OVFEM_DEFINE_LAUNCHERS(PATH_FP64, 8, 0)
OVFEM_DEFINE_LAUNCHERS(PATH_FP64, 8, 1)
OVFEM_DEFINE_LAUNCHERS(PATH_FP64SF, 8, 0)
OVFEM_DEFINE_LAUNCHERS(PATH_FP64SF, 8, 1)

}  // namespace ovfem
