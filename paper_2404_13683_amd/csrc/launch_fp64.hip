// Kernel instantiations: PATH_FP64, 8, 0; PATH_FP64, 8, 1; PATH_FP64SF, 8, 0.
#include "launch_impl.hpp"

namespace ovfem {

OVFEM_DEFINE_LAUNCHERS(PATH_FP64, 8, 0)
OVFEM_DEFINE_LAUNCHERS(PATH_FP64, 8, 1)
OVFEM_DEFINE_LAUNCHERS(PATH_FP64SF, 8, 0)

}  // namespace ovfem
