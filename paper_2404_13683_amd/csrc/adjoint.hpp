// HIP kernel (gfx950) of the per-element gradient terms of the discrete adjoint.
#pragma once

#include "kernels.hpp"

namespace ovfem {

// The two energies w^T K_lam u and w^T K_mu u of one element (h = 1) in the
// sum-factorised form of sf_component: with W, Wh the Walsh coefficients of u and w
// (sf_transform) and f_b = (1/16) q^|b| (q = 3/4 OVFEM, 1/3 trilinear),
//     w^T K_lam u = sum_b f_b tr_b(u) tr_b(w),
//     w^T K_mu u  = sum_b f_b sum_{j not in b} sum_c Wh_c[b+{j}] (W_c[b+{j}] + [c not in b] W_j[b+{c}]),
// since w^T y = sum_{c,S} Wh_c[S] V_c[S] for y_{alpha,c} = sum_S chi_S(alpha) V_c[S].
template <int ELEM>
__device__ inline void sf_energies(const double W[3][8], const double tr[7], const double Wh[3][8],
                                   const double trh[7], double& el, double& em) {
  constexpr double q = ELEM == 1 ? 1.0 / 3.0 : 0.75;
  const double f[3] = {1.0 / 16.0, q / 16.0, q * q / 16.0};
  el = 0.0;
  em = 0.0;
#pragma unroll
  for (int ib = 0; ib < 7; ++ib) {
    const int b = kSfB[ib];
    const int nb = (b & 1) + ((b >> 1) & 1) + ((b >> 2) & 1);
    double sm = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if ((b >> j) & 1) continue;
      const int S = b | (1 << j);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double g = W[c][S];
        if (!((b >> c) & 1)) g += W[j][b | (1 << c)];
        sm = fma(Wh[c][S], g, sm);
      }
    }
    el = fma(f[nb] * tr[ib], trh[ib], el);
    em = fma(f[nb], sm, em);
  }
}

// Tiling of the gradient kernel: 16 x 16 elements per work-group (one per thread), marching
// up through a chunk of element layers with the node planes of u and w staged in LDS.
constexpr int GT = 16;           // elements per tile side
constexpr int GN = GT + 1;       // nodes per staged plane side
constexpr int GPLANE = GN * GN;  // nodes per staged plane

// Per-element gradient terms of the discrete adjoint: for every solid element e,
//     g_lam[e] -= h w_e^T K_lam u_e,   g_mu[e] -= h w_e^T K_mu u_e,
// with u = u^{m-1} (DAMP: the staged (1+b) u^{m-1} - b u^{m-2}, b = beta/dt, as the damped
// step stages it) and w = w^m (the derivative of w^T K u with respect to lam_e, mu_e, from
// K_e = h (lam_e K_lam + mu_e K_mu)).  The energies are formed sum-factorised (sf_energies:
// about 300 flops per element instead of the 2304 of two dense 24 x 24 products).
// Work-group (tx, ty, chunk) owns elements 16 tx .. 16 tx + 15 by 16 ty .. 16 ty + 15 of
// layers chunk * zchunk .. + zchunk - 1; each node of a plane is read from memory once per
// work-group (coalesced rows of 17 nodes) into a two-plane LDS ring ([component][node]),
// and each thread reads its element's 8 corners from there.  Each element's sums are
// private to its thread, so the accumulation order is fixed.  ELEM: 0 OVFEM, 1 trilinear.
template <int ELEM, bool DAMP>
__global__ void __launch_bounds__(GT * GT) ovfem_gradient_kernel(Geom g, int zchunk, double h, const double* mat,
                                                                  const double* u, const double* u2, double b,
                                                                  const double* w, double* g_lam, double* g_mu) {
  __shared__ double su[2][3 * GPLANE], sw[2][3 * GPLANE];
  const int tiles_x = (g.nx + GT - 1) / GT, tiles_y = (g.ny + GT - 1) / GT;
  const int tile = blockIdx.x % (tiles_x * tiles_y), chunk = blockIdx.x / (tiles_x * tiles_y);
  const int x0 = GT * (tile % tiles_x), y0 = GT * (tile / tiles_x);
  const int z0 = chunk * zchunk, z1 = min(g.nz, z0 + zchunk);
  const int tid = threadIdx.x, ex = tid % GT, ey = tid / GT;
  const int X = x0 + ex, Y = y0 + ey;
  const bool mine = X < g.nx && Y < g.ny;
  const size_t plane = (size_t)(g.nx + 1) * (g.ny + 1);

  // node plane Zn of the tile into ring slot `slot` (0 outside the grid)
  auto stage = [&](int slot, int Zn) {
    for (int k = tid; k < GPLANE; k += GT * GT) {
      const int gx = x0 + k % GN, gy = y0 + k / GN;
      double uv[3] = {0.0, 0.0, 0.0}, wv[3] = {0.0, 0.0, 0.0};
      if (gx <= g.nx && gy <= g.ny) {
        const size_t n = 3 * ((size_t)Zn * plane + (size_t)gy * (g.nx + 1) + gx);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double x = u[n + c];
          uv[c] = DAMP ? fma(b, x - u2[n + c], x) : x;
          wv[c] = w[n + c];
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        su[slot][c * GPLANE + k] = uv[c];
        sw[slot][c * GPLANE + k] = wv[c];
      }
    }
  };

  if (z0 >= z1) return;  // the whole work-group: no barrier is skipped by part of it
  stage(0, z0);
  for (int Z = z0; Z < z1; ++Z) {
    const int bot = (Z - z0) & 1, top = bot ^ 1;
    stage(top, Z + 1);
    __syncthreads();
    if (mine) {
      const size_t e = (size_t)Z * g.nx * g.ny + (size_t)Y * g.nx + X;
      const double2 m = reinterpret_cast<const double2*>(mat)[e];
      if (m.x != 0.0 || m.y != 0.0) {  // not a removed voxel
        double ue[24], we[24];
#pragma unroll
        for (int alpha = 0; alpha < 8; ++alpha) {
          const int slot = (alpha >> 2) ? top : bot;
          const int k = (ex + (alpha & 1)) + GN * (ey + ((alpha >> 1) & 1));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            ue[3 * alpha + c] = su[slot][c * GPLANE + k];
            we[3 * alpha + c] = sw[slot][c * GPLANE + k];
          }
        }
        double Wu[3][8], tru[7], Ww[3][8], trw[7];
        sf_transform(ue, Wu, tru);
        sf_transform(we, Ww, trw);
        double gl, gm;
        sf_energies<ELEM>(Wu, tru, Ww, trw, gl, gm);
        g_lam[e] -= h * gl;
        g_mu[e] -= h * gm;
      }
    }
    __syncthreads();  // slot `bot` is staged again next layer
  }
}

}  // namespace ovfem
