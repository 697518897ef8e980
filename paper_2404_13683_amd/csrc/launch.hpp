// Launchers of the stepper kernels, one explicit instantiation per element-product
// path (and digit stage count) in its own translation unit (launch_*.hip), so that the
// kernels compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ovfem {

// One record of KArgs (A.n_units shots at fixed strides): one work-group per tile and
// shot.  ty: tile height in element rows (16 or 32, Tile<TY>); mode: MODE_STEP or
// MODE_MATVEC; damp: Rayleigh-damped step.
template <int PATH, int M, int ELEM>
void launch_tiles(int ty, int mode, bool damp, const KArgs& A, const long long* base, long long step,
                  hipStream_t stream);

// A work list of units with their own records; grid < total selects the strided kernel.
template <int PATH, int M, int ELEM>
void launch_list(int ty, bool damp, int grid, const KArgs* units, const int* begin, int n_units, int total,
                 const long long* base, long long step, hipStream_t stream);

#define OVFEM_DECLARE_LAUNCHERS(PATH, M, ELEM)                                                                   \
  extern template void launch_tiles<PATH, M, ELEM>(int, int, bool, const KArgs&, const long long*, long long,    \
                                                   hipStream_t);                                                \
  extern template void launch_list<PATH, M, ELEM>(int, bool, int, const KArgs*, const int*, int, int,           \
                                                  const long long*, long long, hipStream_t);

OVFEM_DECLARE_LAUNCHERS(PATH_FP64, 8, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_FP64, 8, 1)
OVFEM_DECLARE_LAUNCHERS(PATH_FP64SF, 8, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_FP64SF, 8, 1)
OVFEM_DECLARE_LAUNCHERS(PATH_BF16, 8, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_INT8, 4, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_INT8, 5, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_INT8, 6, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_INT8, 7, 0)
OVFEM_DECLARE_LAUNCHERS(PATH_INT8, 8, 0)

}  // namespace ovfem
