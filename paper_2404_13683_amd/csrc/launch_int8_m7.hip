// Kernel instantiations: PATH_INT8, 7, 0.
#include "launch_impl.hpp"

namespace ovfem {

OVFEM_DEFINE_LAUNCHERS(PATH_INT8, 7, 0)

}  // namespace ovfem
