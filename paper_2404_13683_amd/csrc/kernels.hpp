// HIP kernels (gfx950) of the OVFEM voxel stepper.
//
// One work-group of 256 threads owns a tile of 15 x 15 node columns and a chunk of
// `tz` node planes.  It marches up through the chunk one element layer at a time.
// For element layer k it stages node plane k+1 in LDS (plane k is already there),
// computes the 16 x 16 elements whose corners touch the owned nodes (one halo
// element on each side), keeps each element's contribution to plane k+1 in
// registers, and sums the four in-plane contributions to every owned node of plane
// k.  Plane k is then complete (element layers k-1 and k), so the central-difference
// update of Sec. 2, Eq. (3) runs for it at once:
//     u^{n+1} = 2 u^n - u^{n-1} + dt^2 m^{-1} (F^n - (K u^n))   (zero where m^{-1} = 0).
// Every node is summed by exactly one thread in a fixed order, so results are
// bitwise reproducible (no atomics).
//
// Element products, K_e u_e = h lam_e K_lam u_e + h mu_e K_mu u_e with integer
// AL = 256 K_lam, AM = 128 K_mu (refmat.hpp):
//   * FP64 path: one thread per element, dense 24 x 24 products in FP64 with the
//     integer matrices as compile-time constants (the paper's "OVFEM FP64").
//   * INT8 path (Sec. 2, Eqs. (10)-(17), reworked for CDNA4): u is written as
//     2^(E-62) q with q an integer, |q| <= 2^62, under one power-of-two exponent E per
//     tile (the paper scales per element by s_e; a shared exponent lets a node's
//     digits be computed once and reused by its 8 elements, and the extra bits keep
//     every value within 2^9 of the tile maximum exact).  q is split into M = 8
//     balanced base-256 digits d_j in [-128, 127] (the paper uses 8 sign-magnitude
//     base-128 digits of a 56-bit integer).  The 48 x 24 matrix [AL; AM] times the
//     digit panel of 16 elements runs on v_mfma_i32_16x16x32_i8.  Digits are taken
//     pairwise from the top, C = A d_hi, C <<= 8, C += A d_lo, which stays below
//     2^31 since |C| <= 384 * 128 * 257; the four group results are recombined in
//     FP64 (Horner with factor 2^16), then scaled by h lam_e / 256 * 2^(E-62) and
//     h mu_e / 128 * 2^(E-62).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "refmat.hpp"

namespace ovfem {

constexpr int TE = 16;        // element columns per tile side
constexpr int TN = TE - 1;    // owned node columns per tile side
constexpr int PN = TE + 1;    // node columns per staged plane side
constexpr int NTHR = 256;     // threads per work-group
constexpr int NDIG = 8;       // balanced base-256 digits per value
constexpr int QBITS = 62;     // fraction bits of q under the tile exponent
constexpr int PP = 18;        // padded pitch (dwords) of a digit row
constexpr int DPLANE = PN * NDIG * PP;  // dwords per staged digit plane
constexpr int FPLANE = 3 * PN * PN;     // doubles per staged FP64 plane
constexpr int EXP_NONE = -1000000;      // exponent of an all-zero tile

static_assert(kMaxRowAbs * 128 * 257 < 2147483647, "two-digit INT32 Horner group must not overflow");

enum : int { MODE_STEP = 0, MODE_MATVEC = 1 };
enum : int { PATH_FP64 = 0, PATH_INT8 = 1 };

typedef int v4i __attribute__((ext_vector_type(4)));

struct Geom {
  int nx, ny, nz;       // elements per axis
  int tz;               // node planes per chunk
  int tiles_x, tiles_y, chunks;
  int n_wg;
};

struct KArgs {
  Geom g;
  const double* u;        // u^n, [node][3]
  double* uprev_next;     // in: u^{n-1}; out: u^{n+1} (same array)
  double* ku;             // MODE_MATVEC output K u, [node][3]
  const double* lam_s;    // h lam / 256 per element (0 for removed voxels)
  const double* mu_s;     // h mu / 128 per element
  const double* acoef;    // dt^2 / m per node, 0 where the node does not move
  const int* exp_in;      // per tile: exponent e with max |u^n| < 2^e (INT8 path)
  int* exp_out;           // per tile: same for u^{n+1} (MODE_STEP)
  const uint64_t* alane;  // INT8 A operands, [3 row tiles][64 lanes]
  const int* src_ptr;     // [n_wg + 1] CSR of sources per tile
  const int* src_node;    // node id of each listed source
  const int* src_comp;    // component
  const int* src_row;     // row of the wavelet table
  const double* wavelet;  // [n_src][src_nt]
  const int* rec_ptr;     // [n_wg + 1] CSR of receivers per tile
  const int* rec_node;
  const int* rec_idx;     // receiver index
  double* traces;         // [rec][3][rec_nt]
  int src_nt, rec_nt;
  long long step;         // index n of the step being taken
};

// Logical tile of this work-group.  Work-groups are dealt to the 8 XCDs round-robin
// in blockIdx order; remap so that each XCD gets a contiguous run of tiles and
// neighbouring tiles share that XCD's L2.
__device__ inline int logical_tile(int b, int n_wg) {
  const int xcd = b & 7, slot = b >> 3, n8 = n_wg >> 3, rem = n_wg & 7;
  return xcd < rem ? xcd * (n8 + 1) + slot : rem * (n8 + 1) + (xcd - rem) * n8 + slot;
}

__device__ inline long long node_index(const Geom& g, int X, int Y, int Z) {
  return (long long)X + (long long)(g.nx + 1) * ((long long)Y + (long long)(g.ny + 1) * Z);
}

struct D3 {
  double v[3];
};

// The three components of node (X, Y, Z) of v, zero outside the grid.
__device__ inline D3 load_node(const Geom& g, const double* v, int X, int Y, int Z) {
  D3 r = {{0.0, 0.0, 0.0}};
  if (X >= 0 && Y >= 0 && Z >= 0 && X <= g.nx && Y <= g.ny && Z <= g.nz) {
    const double* p = v + 3 * node_index(g, X, Y, Z);
    r.v[0] = p[0];
    r.v[1] = p[1];
    r.v[2] = p[2];
  }
  return r;
}

// Eight balanced base-256 digits of q = rint(u 2^(62-E)) for the three components,
// packed per digit as bytes (c0, c1, c2, 0): the B-operand layout of the MFMA.
// (lam_s, mu_s) of element (X, Y, Z), zero outside the grid.
__device__ inline D3 load_material(const Geom& g, const double* lam_s, const double* mu_s, int X, int Y, int Z) {
  D3 r = {{0.0, 0.0, 0.0}};
  if (X >= 0 && Y >= 0 && Z >= 0 && X < g.nx && Y < g.ny && Z < g.nz) {
    const long long e = (long long)X + (long long)g.nx * ((long long)Y + (long long)g.ny * Z);
    r.v[0] = lam_s[e];
    r.v[1] = mu_s[e];
  }
  return r;
}

struct DigitWords {
  uint32_t w[NDIG];
};

__device__ inline DigitWords digit_words(const D3& u, int E) {
  uint32_t lo[3], hi[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double x = rint(ldexp(u.v[c], QBITS - E));     // |x| <= 2^62, exact integer
    const double hd = floor(x * 0x1p-32);                 // exact, |hd| <= 2^30
    const uint32_t lo_u = (uint32_t)fma(hd, -0x1p32, x);  // in [0, 2^32), exact
    const uint64_t q = ((uint64_t)(uint32_t)(int)hd << 32) | lo_u;  // two's complement
    // q + sum_j 128 * 256^j (mod 2^64) has the digits (d_j + 128) as its bytes
    const uint64_t d = q + 0x8080808080808080ull;
    lo[c] = (uint32_t)d ^ 0x80808080u;
    hi[c] = (uint32_t)(d >> 32) ^ 0x80808080u;
  }
  DigitWords r;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int sh = 8 * j;
    r.w[j] = ((lo[0] >> sh) & 0xffu) | (((lo[1] >> sh) & 0xffu) << 8) | (((lo[2] >> sh) & 0xffu) << 16);
  }
#pragma unroll
  for (int j = 4; j < NDIG; ++j) {
    const int sh = 8 * (j - 4);
    r.w[j] = ((hi[0] >> sh) & 0xffu) | (((hi[1] >> sh) & 0xffu) << 8) | (((hi[2] >> sh) & 0xffu) << 16);
  }
  return r;
}

// Per-element FP64 product: y = lam_s AL ue + mu_s AM ue.
__device__ inline void element_fp64(const double ue[24], double lam_s, double mu_s, double y[24]) {
#pragma unroll
  for (int m = 0; m < 24; ++m) {
    double sl = 0.0, sm = 0.0;
#pragma unroll
    for (int n = 0; n < 24; ++n) {
      sl = fma((double)kRef.AL[m][n], ue[n], sl);
      sm = fma((double)kRef.AM[m][n], ue[n], sm);
    }
    y[m] = lam_s * sl + mu_s * sm;
  }
}

// Wave-wide max of a non-negative double.
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Work-group max of |u| over owned nodes -> tile exponent (shared by the stepper
// and the exponent initialisation kernel).
__device__ inline void write_tile_exponent(double local_max, int* dst, double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  local_max = wave_max(local_max);
  if (lane == 0) red[w] = local_max;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    int e = EXP_NONE;
    if (m > 0.0) frexp(m, &e);  // m < 2^e
    *dst = e;
  }
}

template <int PATH, int MODE>
__global__ void __launch_bounds__(NTHR) ovfem_layer_kernel(KArgs A) {
  const Geom& g = A.g;
  const int wg = logical_tile(blockIdx.x, g.n_wg);
  const int tx = wg % g.tiles_x, ty = (wg / g.tiles_x) % g.tiles_y, tzc = wg / (g.tiles_x * g.tiles_y);
  const int x0 = tx * TN, y0 = ty * TN, z0 = tzc * g.tz;
  const int z1 = min(z0 + g.tz, g.nz + 1);  // owned planes [z0, z1)
  const int t = threadIdx.x;
  const int ta = t & 15, tb = t >> 4;       // element column (ta, tb) / main staged node (ta+1, tb+1)

  __shared__ double acc[4 * 3 * TE * TE];                  // [c2][c][b][a] in-plane corner sums
  __shared__ double red[4];
  // staged planes: FP64 values or INT8 digit words, two slots
  constexpr int RING_BYTES = PATH == PATH_FP64 ? 2 * FPLANE * 8 : 2 * DPLANE * 4;
  __shared__ __attribute__((aligned(16))) unsigned char ring_raw[RING_BYTES];
  __shared__ double mat[PATH == PATH_INT8 ? 2 * TE * TE : 2];  // INT8: [b][a] (lam_s, mu_s)
  double* ringf = reinterpret_cast<double*>(ring_raw);
  uint32_t* ringd = reinterpret_cast<uint32_t*>(ring_raw);

  // ---- tile exponent (INT8): max over the 27 neighbouring tiles that own the staged nodes
  int E = 0;
  if (PATH == PATH_INT8) {
    int e = EXP_NONE;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int X = tx + dx, Y = ty + dy, Z = tzc + dz;
          if (X >= 0 && Y >= 0 && Z >= 0 && X < g.tiles_x && Y < g.tiles_y && Z < g.chunks)
            e = max(e, A.exp_in[X + g.tiles_x * (Y + g.tiles_y * Z)]);
        }
    E = e == EXP_NONE ? 0 : e;
  }

  // INT8 operands: lane's A fragments for the three 16-row tiles
  const int lane = t & 63, wave = t >> 6;
  uint64_t a_frag[3] = {0, 0, 0};
  if (PATH == PATH_INT8) {
    a_frag[0] = A.alane[lane];
    a_frag[1] = A.alane[64 + lane];
    a_frag[2] = A.alane[128 + lane];
  }

  // staged node positions: main node (ta+1, tb+1); threads 0..32 also stage a halo node
  const int mp = ta + 1, mq = tb + 1;
  const int xp = t < 17 ? t : 0, xq = t < 17 ? 0 : t - 16;  // (p, q) of the extra node
  const bool has_extra = t < 33;
  const bool owner = ta < TN && tb < TN;  // owns node (ta+1, tb+1) = (x0+ta, y0+tb)
  const int OX = x0 + ta, OY = y0 + tb;
  const bool owner_in = owner && OX <= g.nx && OY <= g.ny;

  // register pipeline of the main node's u^n (plane rel r = Z - (z0-1))
  D3 u_main_next = {{0.0, 0.0, 0.0}}, u_extra_next = {{0.0, 0.0, 0.0}};
  D3 u_own_bot = {{0.0, 0.0, 0.0}}, u_own_top = {{0.0, 0.0, 0.0}};
  double top_prev[12];  // FP64: this element's contribution to the plane above (4 corners x 3)
  double top_prev8[4][3];
#pragma unroll
  for (int i = 0; i < 12; ++i) top_prev[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) top_prev8[i][0] = top_prev8[i][1] = top_prev8[i][2] = 0.0;
  D3 mat_next = {{0.0, 0.0, 0.0}};  // (lam_s, mu_s) of element (ta, tb) of the next layer
  double tile_max = 0.0;

  const int nrel = z1 - z0 + 2;  // staged planes z0-1 .. z1
  auto fetch = [&](int rel) {
    const int Z = z0 - 1 + rel;
    u_main_next = load_node(g, A.u, x0 - 1 + mp, y0 - 1 + mq, Z);
    if (has_extra) u_extra_next = load_node(g, A.u, x0 - 1 + xp, y0 - 1 + xq, Z);
  };
  auto stage = [&](int slot) {
    if (PATH == PATH_FP64) {
      double* P = ringf + slot * FPLANE;
#pragma unroll
      for (int c = 0; c < 3; ++c) P[(c * PN + mq) * PN + mp] = u_main_next.v[c];
      if (has_extra)
#pragma unroll
        for (int c = 0; c < 3; ++c) P[(c * PN + xq) * PN + xp] = u_extra_next.v[c];
    } else {
      uint32_t* P = ringd + slot * DPLANE;
      const DigitWords w = digit_words(u_main_next, E);
#pragma unroll
      for (int j = 0; j < NDIG; ++j) P[(mq * NDIG + j) * PP + mp] = w.w[j];
      if (has_extra) {
        const DigitWords wx = digit_words(u_extra_next, E);
#pragma unroll
        for (int j = 0; j < NDIG; ++j) P[(xq * NDIG + j) * PP + xp] = wx.w[j];
      }
    }
  };

  // prologue: plane rel 0 staged, plane rel 1 in registers
  fetch(0);
  stage(0);
  fetch(1);
  mat_next = load_material(g, A.lam_s, A.mu_s, x0 - 1 + ta, y0 - 1 + tb, z0 - 1);

  for (int it = 0; it + 1 < nrel; ++it) {
    // element layer k = z0 - 1 + it uses planes rel it (slot it&1) and rel it+1
    const int k = z0 - 1 + it;
    const int bot = it & 1, top = (it + 1) & 1;
    u_own_bot = u_own_top;
    u_own_top = u_main_next;
    stage(top);
    const double lam_e = mat_next.v[0], mu_e = mat_next.v[1];
    if (PATH == PATH_INT8) {
      mat[2 * t] = lam_e;
      mat[2 * t + 1] = mu_e;
    }
    if (it + 2 < nrel) fetch(it + 2);
    if (it + 2 < nrel) mat_next = load_material(g, A.lam_s, A.mu_s, x0 - 1 + ta, y0 - 1 + tb, k + 1);
    // owned plane rel it (Z = k) update operands
    const int Z = k;
    const bool do_node = it >= 1 && owner_in;
    long long nid = 0;
    double up[3] = {0, 0, 0}, ac = 0.0;
    if (do_node) {
      nid = node_index(g, OX, OY, Z);
      if (MODE == MODE_STEP) {
        const double* pp = A.uprev_next + 3 * nid;
        up[0] = pp[0];
        up[1] = pp[1];
        up[2] = pp[2];
        ac = A.acoef[nid];
      }
    }
    __syncthreads();

    // ---- element layer k
    if (PATH == PATH_FP64) {
      const double* Pb = ringf + bot * FPLANE;
      const double* Pt = ringf + top * FPLANE;
      double ue[24];
#pragma unroll
      for (int alpha = 0; alpha < 8; ++alpha) {
        const int di = alpha & 1, dj = (alpha >> 1) & 1, dk = alpha >> 2;
        const double* P = dk ? Pt : Pb;
#pragma unroll
        for (int c = 0; c < 3; ++c) ue[3 * alpha + c] = P[(c * PN + tb + dj) * PN + ta + di];
      }
      double y[24];
      element_fp64(ue, lam_e, mu_e, y);
#pragma unroll
      for (int c2 = 0; c2 < 4; ++c2)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          acc[((c2 * 3 + c) * TE + tb) * TE + ta] = y[3 * c2 + c] + top_prev[3 * c2 + c];
          top_prev[3 * c2 + c] = y[3 * (c2 + 4) + c];
        }
    } else {
      const int ja = lane & 15, G = lane >> 4;
      const uint32_t* Pin = ringd + ((G >> 1) ? top : bot) * DPLANE;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int b = 4 * wave + tt;
        const uint32_t* P = Pin + (b + (G & 1)) * NDIG * PP + ja;
        uint64_t B[NDIG];
#pragma unroll
        for (int j = 0; j < NDIG; ++j) B[j] = (uint64_t)P[j * PP] | ((uint64_t)P[j * PP + 1] << 32);
        double R[12];
#pragma unroll
        for (int r = 0; r < 12; ++r) R[r] = 0.0;
        // digit pairs from the top: (7,6), (5,4), (3,2), (1,0)
#pragma unroll
        for (int pr = 3; pr >= 0; --pr) {
          const int jh = 2 * pr + 1, jl = 2 * pr;
          const v4i z = {0, 0, 0, 0};
          v4i c0 = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)a_frag[0], (long)B[jh], z, 0, 0, 0);
          v4i c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)a_frag[1], (long)B[jh], z, 0, 0, 0);
          v4i c2 = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)a_frag[2], (long)B[jh], z, 0, 0, 0);
          c0 = c0 << 8;
          c1 = c1 << 8;
          c2 = c2 << 8;
          c0 = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)a_frag[0], (long)B[jl], c0, 0, 0, 0);
          c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)a_frag[1], (long)B[jl], c1, 0, 0, 0);
          c2 = __builtin_amdgcn_mfma_i32_16x16x32_i8((long)a_frag[2], (long)B[jl], c2, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            R[r] = fma(R[r], 65536.0, (double)c0[r]);
            R[4 + r] = fma(R[4 + r], 65536.0, (double)c1[r]);
            R[8 + r] = fma(R[8 + r], 65536.0, (double)c2[r]);
          }
        }
        // output s = 4 * tile + reg: s < 6 from AL, s >= 6 from AM; dk = (s % 6) / 3, c = s % 3
        const double sl = ldexp(mat[2 * (b * TE + ja)], E - QBITS);
        const double sm = ldexp(mat[2 * (b * TE + ja) + 1], E - QBITS);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double ybot = R[c] * sl + R[6 + c] * sm;
          const double ytop = R[3 + c] * sl + R[9 + c] * sm;
          acc[((G * 3 + c) * TE + b) * TE + ja] = ybot + top_prev8[tt][c];
          top_prev8[tt][c] = ytop;
        }
        __builtin_amdgcn_sched_barrier(0);  // keep tiles apart: bounds live registers
      }
    }
    __syncthreads();

    // ---- node phase for plane Z = k (owned when it >= 1)
    if (do_node) {
      double f[3];
      const int a = ta, b = tb;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        f[c] = acc[((3 * 3 + c) * TE + b) * TE + a] + acc[((2 * 3 + c) * TE + b) * TE + a + 1] +
               acc[((1 * 3 + c) * TE + b + 1) * TE + a] + acc[((0 * 3 + c) * TE + b + 1) * TE + a + 1];
      if (MODE == MODE_MATVEC) {
        double* o = A.ku + 3 * nid;
        o[0] = f[0];
        o[1] = f[1];
        o[2] = f[2];
      } else {
        double F[3] = {0.0, 0.0, 0.0};
        const int s0 = A.src_ptr[wg], s1 = A.src_ptr[wg + 1];
        for (int s = s0; s < s1; ++s)
          if (A.src_node[s] == (int)nid && A.step < A.src_nt) {
            const double w = A.wavelet[(long long)A.src_row[s] * A.src_nt + A.step];
            const int sc = A.src_comp[s];
            F[0] += sc == 0 ? w : 0.0;
            F[1] += sc == 1 ? w : 0.0;
            F[2] += sc == 2 ? w : 0.0;
          }
        double un[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
          un[c] = ac > 0.0 ? 2.0 * u_own_bot.v[c] - up[c] + ac * (F[c] - f[c]) : 0.0;
        double* o = A.uprev_next + 3 * nid;
        o[0] = un[0];
        o[1] = un[1];
        o[2] = un[2];
        tile_max = fmax(tile_max, fmax(fabs(un[0]), fmax(fabs(un[1]), fabs(un[2]))));
        const int r0 = A.rec_ptr[wg], r1 = A.rec_ptr[wg + 1];
        for (int r = r0; r < r1; ++r)
          if (A.rec_node[r] == (int)nid && A.step < A.rec_nt) {
            double* tr = A.traces + (long long)A.rec_idx[r] * 3 * A.rec_nt + A.step;
            tr[0] = un[0];
            tr[A.rec_nt] = un[1];
            tr[2 * A.rec_nt] = un[2];
          }
      }
    }
  }
  if (MODE == MODE_STEP) write_tile_exponent(tile_max, A.exp_out + wg, red);
}

// Tile exponents of an arbitrary nodal vector (same tiling as the stepper).
__global__ void __launch_bounds__(NTHR) ovfem_exponent_kernel(Geom g, const double* u, int* exp_out) {
  __shared__ double red[4];
  const int wg = blockIdx.x;
  const int tx = wg % g.tiles_x, ty = (wg / g.tiles_x) % g.tiles_y, tzc = wg / (g.tiles_x * g.tiles_y);
  const int t = threadIdx.x, ta = t & 15, tb = t >> 4;
  const int X = tx * TN + ta, Y = ty * TN + tb;
  const int z0 = tzc * g.tz, z1 = min(z0 + g.tz, g.nz + 1);
  double m = 0.0;
  if (ta < TN && tb < TN && X <= g.nx && Y <= g.ny)
    for (int Z = z0; Z < z1; ++Z) {
      const double* p = u + 3 * node_index(g, X, Y, Z);
      m = fmax(m, fmax(fabs(p[0]), fmax(fabs(p[1]), fabs(p[2]))));
    }
  write_tile_exponent(m, exp_out + wg, red);
}

}  // namespace ovfem
