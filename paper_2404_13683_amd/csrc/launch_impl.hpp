// Definitions of the launchers declared in launch.hpp (included by the launch_*.hip
// translation units only).
#pragma once

#include "launch.hpp"

namespace ovfem {

template <int PATH, int M, int ELEM, int TY>
void launch_tiles_ty(int mode, bool damp, const KArgs& A, const long long* base, long long step, hipStream_t stream) {
  const dim3 grid(A.g.n_wg * (A.n_units > 1 ? A.n_units : 1)), block(Tile<TY>::THREADS);
  if (mode == MODE_MATVEC)
    ovfem_layer_kernel<PATH, MODE_MATVEC, M, false, ELEM, TY><<<grid, block, 0, stream>>>(A, base, step);
  else if (damp)
    ovfem_layer_kernel<PATH, MODE_STEP, M, true, ELEM, TY><<<grid, block, 0, stream>>>(A, base, step);
  else
    ovfem_layer_kernel<PATH, MODE_STEP, M, false, ELEM, TY><<<grid, block, 0, stream>>>(A, base, step);
}

template <int PATH, int M, int ELEM>
void launch_tiles(int ty, int mode, bool damp, const KArgs& A, const long long* base, long long step,
                  hipStream_t stream) {
  if (ty == 32)
    launch_tiles_ty<PATH, M, ELEM, 32>(mode, damp, A, base, step, stream);
  else
    launch_tiles_ty<PATH, M, ELEM, 16>(mode, damp, A, base, step, stream);
}

template <int PATH, int M, int ELEM, int TY>
void launch_list_ty(bool damp, int grid, const KArgs* units, const int* begin, int n_units, int total,
                    const long long* base, long long step, hipStream_t stream) {
  const dim3 g(grid), block(Tile<TY>::THREADS);
  if (grid >= total) {
    if (damp)
      ovfem_batch_kernel<PATH, MODE_STEP, M, true, ELEM, TY><<<g, block, 0, stream>>>(units, begin, n_units, total,
                                                                                     base, step);
    else
      ovfem_batch_kernel<PATH, MODE_STEP, M, false, ELEM, TY><<<g, block, 0, stream>>>(units, begin, n_units, total,
                                                                                      base, step);
  } else {
    if (damp)
      ovfem_batch_strided_kernel<PATH, MODE_STEP, M, true, ELEM, TY><<<g, block, 0, stream>>>(units, begin, n_units,
                                                                                             total, base, step);
    else
      ovfem_batch_strided_kernel<PATH, MODE_STEP, M, false, ELEM, TY><<<g, block, 0, stream>>>(units, begin, n_units,
                                                                                              total, base, step);
  }
}

template <int PATH, int M, int ELEM>
void launch_list(int ty, bool damp, int grid, const KArgs* units, const int* begin, int n_units, int total,
                 const long long* base, long long step, hipStream_t stream) {
  if (ty == 32)
    launch_list_ty<PATH, M, ELEM, 32>(damp, grid, units, begin, n_units, total, base, step, stream);
  else
    launch_list_ty<PATH, M, ELEM, 16>(damp, grid, units, begin, n_units, total, base, step, stream);
}

#define OVFEM_DEFINE_LAUNCHERS(PATH, M, ELEM)                                                                 \
  template void launch_tiles<PATH, M, ELEM>(int, int, bool, const KArgs&, const long long*, long long,       \
                                            hipStream_t);                                                   \
  template void launch_list<PATH, M, ELEM>(int, bool, int, const KArgs*, const int*, int, int, const long long*, \
                                           long long, hipStream_t);

}  // namespace ovfem
