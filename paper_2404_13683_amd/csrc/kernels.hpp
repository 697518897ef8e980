// HIP kernels (gfx950) of the OVFEM voxel stepper.
//
// Work decomposition.  A work-group of 256 threads (4 waves) owns a tile of 15 x 15
// node columns and a chunk of `tz` node planes, and marches up through the chunk one
// element layer at a time.  For element layer k it stages node plane k+1 in LDS
// (plane k is already there), computes the 16 x 16 elements whose corners touch the
// owned nodes (one halo element on each side), keeps each element's contribution to
// plane k+1 in registers for the next layer, and forms the in-plane sums of the
// contributions to plane k.  Plane k is then complete (element layers k-1 and k) and
// the central-difference update of Sec. 2, Eq. (3) runs for it at once:
//     u^{n+1} = 2 u^n - u^{n-1} + dt^2 m^{-1} (F^n - (K u^n))   (zero where m^{-1} = 0),
// or its Rayleigh-damped form (DAMP kernels; see KArgs).  Every owned node is updated
// by one thread; the in-plane sums are formed in LDS with a fixed set of addends per
// entry (a store, then at most one add of a second term: two-term sums commute
// exactly), so results are bitwise reproducible.  No global atomics.
//
// Element products, K_e u_e = h lam_e K_lam u_e + h mu_e K_mu u_e with the integer
// matrices AL = 256 K_lam, AM = 128 K_mu (refmat.hpp):
//   * FP64 path: one thread per element, dense 24 x 24 products in FP64 with the
//     integer matrices as compile-time constants (the paper's "OVFEM FP64").
//   * INT8 paths (Sec. 2, Eqs. (10)-(17), reworked for CDNA4).  u is written as
//     2^(S-QB) q, q = u 2^(QB-S) rounded to the nearest integer, |q| <= 2^QB, under
//     one power-of-two exponent S per element layer of the work-group (the paper
//     scales each element by its own s_e; an exponent shared by the 17 x 17 x 2
//     staged nodes of a layer lets a node's slices be computed once for the 4
//     elements of the layer that touch it).  2^S is the smallest power of two above
//     every staged value with S a multiple of EXP_QUANT, taken from the staged values
//     themselves (key_exponent); a node plane is staged again only when the next
//     layer's S differs.  q is split into M balanced base-256 digits d_j in [-128, 127],
//     QB = 8M - 2 (M = 8 by default: 62 bits, so every entry is represented to
//     2^(S-63) absolutely, at least 2^-59 relative to the layer maximum; the paper: 8
//     sign-magnitude base-128 digits of a 56-bit integer), and the digit
//     products with the 48 x 24 integer matrix [AL; AM] run on the matrix cores, digits
//     taken pairwise from the top.  PATH_INT8 uses v_mfma_i32_16x16x32_i8:
//     C = A d_hi, C <<= 8, C += A d_lo, exact in INT32 since
//     |C| <= 384 * 128 * 257 < 2^31 (the paper flushes INT32 every 3 stages).
//     PATH_BF16 (M = 8) uses v_mfma_f32_16x16x32_bf16 with A (256 d_hi) + A (d_lo + 128)
//     in one FP32 accumulator: every operand is an integer of at most 8 significant
//     bits (exact in bf16) and every partial sum an integer below
//     384 * 128 * 256 + 384 * 255 < 2^24 (exact in FP32); the +128 bias drops out
//     because each row of K sums to zero (rigid translations).  Both give the same
//     pair sums, which are recombined in FP64 (Horner with factor 2^16) and scaled by
//     h lam_e / 256 * 2^(S-QB) and h mu_e / 128 * 2^(S-QB).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "refmat.hpp"

namespace ovfem {

constexpr int TE = 16;        // element columns per tile side
constexpr int TN = TE - 1;    // owned node columns per tile side
constexpr int PN = TE + 1;    // node columns per staged plane side
constexpr int NTHR = 256;     // threads per work-group of the one-element-per-thread kernels
constexpr int NPAIR = 4;      // digit pairs (M = 8 digits)
constexpr int QBITS = 62;     // fraction bits of q under the staging exponent
constexpr int NODE_DW = 16;   // dwords of one staged node: 4 pairs x (hi, lo) x 2 dwords
// digit plane layout [row q][pair p][hi/lo][column x][2 dwords]: the B operand of a
// lane (its element's nodes x and x+1 in one row) is 16 contiguous bytes
constexpr int DROW = NPAIR * 2 * PN * 2;   // dwords per staged digit row
// i8 form with M digits (stages): [row q][digit j][column x] one dword (c0, c1, c2, 0)
// of signed digits.  Rows are padded to 16 (mod 64) dwords and planes to 32 (mod 64),
// so the four 16-lane groups of a B-operand read (two tile rows, two planes) and the
// four 16-thread rows of a staging write fall on disjoint LDS banks.
constexpr int pad_to(int n, int r) { return n + ((r - n % 64) + 64) % 64; }
template <int M>
struct Stages {
  static_assert(M >= 4 && M <= 8, "4 to 8 digit stages");
  static constexpr int QB = 8 * M - 2;         // fraction bits of q: |q| < 2^QB
  static constexpr int NG = (M + 1) / 2;       // digit groups (pairs; the top one single if M is odd)
  static constexpr int ROW = pad_to(M * PN, 16);
  static constexpr int PLANE = pad_to(PN * ROW, 32);
};
// Tile height: TY element rows per work-group (16 or 32), 16 TY threads, TY / 4 waves of
// four tile rows each; TY - 1 owned node rows.  The x extent is TE (the matrix-core columns).
template <int TY>
struct Tile {
  static_assert(TY == 16 || TY == 32, "tile heights of 16 or 32 element rows");
  static constexpr int THREADS = TE * TY;
  static constexpr int WAVES = THREADS / 64;
  static constexpr int NY = TY - 1;                     // owned node rows
  static constexpr int PNY = TY + 1;                    // staged node rows
  static constexpr int EXTRA = PN * PNY - THREADS;      // staged nodes beyond one per thread
  static constexpr int FPLANE = 3 * PN * PNY;           // doubles per staged FP64 plane
  static constexpr int DPLANE = PN * PNY * NODE_DW;     // dwords per staged bf16 digit plane
  template <int M>
  static constexpr int iplane() { return pad_to(PNY * Stages<M>::ROW, 32); }  // dwords per i8 digit plane
  static_assert(EXTRA > 0 && EXTRA <= 64, "the extra staged nodes fit in the last wave");
};
// Staging exponent of the INT8 paths: S is the exact exponent of the layer's staged
// maximum rounded up to a multiple of EXP_QUANT (so a layer shares its neighbour's S, and
// the plane they share is not staged again, unless the maximum moves across a multiple:
// fewer restages for at most EXP_QUANT - 1 bits of the QB), and S >= EXP_FLOOR keeps the
// scale factors h lam / 256 2^(S-QB) normal (values below 2^(EXP_FLOOR-QB-1) round to 0).
constexpr int EXP_FLOOR = -900;
constexpr int EXP_QUANT = 4;
static_assert(EXP_FLOOR % EXP_QUANT == 0 && (EXP_QUANT & (EXP_QUANT - 1)) == 0, "staging exponent quantum");

static_assert(kMaxRowAbs * 128 * 256 + kMaxRowAbs * 255 < (1 << 24),
              "digit-pair sums must be exact in FP32");
static_assert((long long)kMaxRowAbs * 128 * 257 < 2147483647LL, "digit-pair sums must fit INT32");

enum : int { MODE_STEP = 0, MODE_MATVEC = 1 };
// PATH_INT8: digits on i8 matrix cores, INT32 accumulation with a shift per pair;
// PATH_BF16: digit pairs on bf16 matrix cores, exact FP32 accumulation.
// PATH_FP64SF: the element product in FP64, sum-factorised (sf_transform, sf_component).
enum : int { PATH_FP64 = 0, PATH_INT8 = 1, PATH_BF16 = 2, PATH_FP64SF = 3 };
constexpr bool is_f64_path(int p) { return p == PATH_FP64 || p == PATH_FP64SF; }
// work-groups per CU named in the launch bounds: the i8 kernels are held to 128 registers
// (four waves per SIMD), the bf16 ones to 256 / 2, the FP64 ones left free
constexpr int groups_per_cu(int path, int ty) {
  return is_f64_path(path) ? 1 : (path == PATH_INT8 ? (ty == 16 ? 4 : 2) : (ty == 16 ? 2 : 1));
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

struct Geom {
  int nx, ny, nz;  // elements per axis
  int tz;          // node planes per chunk
  int tiles_x, tiles_y, chunks;
  int n_wg;
  int ty;          // element rows per tile (Tile<TY>; the kernel's template argument)
};

struct KArgs {
  Geom g;
  const double* u;        // u^n, [node][3]
  const double* uprev;    // u^{n-1}
  double* unext;          // u^{n+1}; may be the same array as uprev (each node is read
                          // and then written by one thread)
  double* ku;             // MODE_MATVEC output K u, [node][3]
  const double* mat;      // [element][2] = (h lam / 256, h mu / 128), 0 for removed voxels
  const double* acoef;    // dt^2 / m per node, 0 where the node does not move
  const v4u* alane;       // INT8 A operands, [3 row tiles][64 lanes] x 8 bf16
  const uint64_t* alane8; // I8 A operands, [3 row tiles][64 lanes] x 8 int8
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
  long long step;         // batch launches: the unit's step offset
  // Rayleigh damping (DAMP kernels only): the product is K w with
  // w = u^n + damp_b (u^n - u^{n-1}), damp_b = beta / dt, and
  // u^{n+1} = damp_c1 u^n - damp_c2 u^{n-1} + acoef (F - K w), with
  // damp_c1 = 2 / (1 + alpha dt / 2), damp_c2 = (1 - alpha dt / 2) / (1 + alpha dt / 2) and
  // acoef = dt^2 / (m (1 + alpha dt / 2)).  unext must then not alias uprev (the halo
  // of u^{n-1} is read by neighbouring work-groups).
  double damp_b, damp_c1, damp_c2;
  // shots of one grid in one launch (ovfem_layer_kernel): n_units units of n_wg tiles,
  // unit v at these element offsets from the pointers above (0 units taken as 1)
  int n_units;
  long long unit_u;    // nodal vectors: u, uprev, unext
  int unit_src;        // src_ptr
  long long unit_tr;   // traces
};

// Logical tile of this work-group.  Work-groups are dealt to the 8 XCDs round-robin
// in blockIdx order; remap so that each XCD gets a contiguous run of tiles and
// neighbouring tiles share that XCD's L2.
__device__ inline int logical_tile(int b, int n_wg) {
  const int xcd = b & 7, slot = b >> 3, n8 = n_wg >> 3, rem = n_wg & 7;
  return xcd < rem ? xcd * (n8 + 1) + slot : rem * (n8 + 1) + (xcd - rem) * n8 + slot;
}

struct D3 {
  double v[3];
};

// A staged node column: in-plane validity and the byte offset of the node within a
// plane of nodal vectors (clamped to node 0 when the column lies outside the grid).
struct NodeRef {
  bool xy_ok;
  uint32_t off;  // byte offset of [node][3] within one plane
};

__device__ inline NodeRef node_ref(const Geom& g, int X, int Y) {
  NodeRef r;
  r.xy_ok = X >= 0 && Y >= 0 && X <= g.nx && Y <= g.ny;
  r.off = r.xy_ok ? 24u * (uint32_t)(X + (g.nx + 1) * Y) : 0u;  // below 2^32 (checked at create)
  return r;
}

// Node of a plane: the load always hits valid memory; values outside the grid are 0.
__device__ inline D3 load_node(const unsigned char* plane, const NodeRef& n, bool z_ok) {
  const double* p = reinterpret_cast<const double*>(plane + n.off);
  const bool ok = n.xy_ok && z_ok;
  D3 r;
  r.v[0] = ok ? p[0] : 0.0;
  r.v[1] = ok ? p[1] : 0.0;
  r.v[2] = ok ? p[2] : 0.0;
  return r;
}

// An element column: validity and the byte offset of [element][2] within one layer.
struct ElemRef {
  bool xy_ok;
  uint32_t off;
};

__device__ inline ElemRef elem_ref(const Geom& g, int X, int Y) {
  ElemRef r;
  r.xy_ok = X >= 0 && Y >= 0 && X < g.nx && Y < g.ny;
  r.off = r.xy_ok ? 16u * (uint32_t)(X + g.nx * Y) : 0u;
  return r;
}

// (h lam / 256, h mu / 128) of an element of a layer, zero outside the grid.
__device__ inline double2 load_material(const unsigned char* layer, const ElemRef& e, bool z_ok) {
  const double2 m = *reinterpret_cast<const double2*>(layer + e.off);
  const bool ok = e.xy_ok && z_ok;
  return make_double2(ok ? m.x : 0.0, ok ? m.y : 0.0);
}

// bf16 words of two floats with at most 8 significant bits (truncation is exact).
__device__ inline uint32_t bf16_pair(float lo, float hi) {
  return __builtin_amdgcn_perm(__float_as_uint(hi), __float_as_uint(lo), 0x07060302u);
}

// q = u 2^(QB-S) rounded to the nearest integer (|u| < 2^S, so |q| <= 2^QB <= 2^62), as
// a two's-complement 64-bit integer.  q = hd 2^32 + lo with hd = floor(q 2^-32) and
// 0 <= lo < 2^32: q is an integer, so both steps are exact and lo converts in range.
template <int QB>
__device__ inline uint64_t quantise(double u, int S) {
  const double x = rint(ldexp(u, QB - S));
  const double hd = floor(x * 0x1p-32);                 // exact, |hd| <= 2^30
  const uint32_t lo_u = (uint32_t)fma(hd, -0x1p32, x);  // exact, in [0, 2^32)
  return ((uint64_t)(uint32_t)(int)hd << 32) | lo_u;
}

// Stage one node's INT8 slices: q = rint(u 2^(62-S)) per component, the biased bytes
// e_j = d_j + 128 of q + sum_j 128 * 256^j, and per digit pair p the bf16 B-operand
// words (c0, c1), (c2, 0) of 256 d_{2p+1} (hi) and of e_{2p} (lo).  dst points at the
// node's first word in its row ([p][hi/lo][x][2] with x stride 2 dwords).
__device__ inline void stage_digits(const D3& u, int S, uint32_t* dst) {
  uint32_t lo[3], hi[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const uint64_t q = quantise<QBITS>(u.v[c], S);
    const uint64_t d = q + 0x8080808080808080ull;        // bytes are d_j + 128
    lo[c] = (uint32_t)d;
    hi[c] = (uint32_t)(d >> 32);
  }
  uint32_t w[NODE_DW];
#pragma unroll
  for (int p = 0; p < NPAIR; ++p) {
    const int bh = (2 * p + 1) & 3, bl = (2 * p) & 3;  // byte positions of the pair
    float fh[3], fl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const uint32_t s = p < 2 ? lo[c] : hi[c];
      fh[c] = fmaf((float)((s >> (8 * bh)) & 0xffu), 256.0f, -32768.0f);  // 256 d_hi, exact
      fl[c] = (float)((s >> (8 * bl)) & 0xffu);                            // d_lo + 128
    }
    w[4 * p + 0] = bf16_pair(fh[0], fh[1]);
    w[4 * p + 1] = __float_as_uint(fh[2]) >> 16;
    w[4 * p + 2] = bf16_pair(fl[0], fl[1]);
    w[4 * p + 3] = __float_as_uint(fl[2]) >> 16;
  }
#pragma unroll
  for (int p = 0; p < NPAIR; ++p)
#pragma unroll
    for (int hl = 0; hl < 2; ++hl) {
      uint2* d2 = reinterpret_cast<uint2*>(dst + (2 * p + hl) * PN * 2);
      *d2 = make_uint2(w[4 * p + 2 * hl], w[4 * p + 2 * hl + 1]);
    }
}

// i8 form of the node staging with M digits: q = rint(u 2^(8M-2-S)), |q| <= 2^(8M-2),
// written as M balanced base-256 digits (the bytes of q + sum_j 128 * 256^j, minus 128;
// the bytes above M are then exactly 128); per digit j the word
// (d_j(c0), d_j(c1), d_j(c2), 0) is written at dst[j * PN].
template <int M>
__device__ inline void stage_digits_i8(const D3& u, int S, uint32_t* dst) {
  constexpr int QB = Stages<M>::QB;
  uint32_t lo[3], hi[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (M <= 4) {
      const int q = (int)rint(ldexp(u.v[c], QB - S));  // |q| <= 2^30
      lo[c] = ((uint32_t)q + 0x80808080u) ^ 0x80808080u;
      hi[c] = 0u;
      continue;
    }
    const uint64_t q = quantise<QB>(u.v[c], S);
    const uint64_t d = q + 0x8080808080808080ull;  // bytes d_j + 128
    lo[c] = (uint32_t)d ^ 0x80808080u;              // bytes d_j (two's complement)
    hi[c] = (uint32_t)(d >> 32) ^ 0x80808080u;
  }
  // digits j, j+1 (bytes sel, sel+1 of one word) from one gather of the c0, c1 bytes:
  // t = (c0 byte sel, c1 byte sel, c0 byte sel+1, c1 byte sel+1), then per digit
  // (t bytes, c2 byte, 0): three byte permutes per two digits
#pragma unroll
  for (int j = 0; j + 1 < M; j += 2) {
    const uint32_t* s = j < 4 ? lo : hi;
    const uint32_t sel = j & 3;
    const uint32_t t = __builtin_amdgcn_perm(s[1], s[0], sel | (sel + 4) << 8 | (sel + 1) << 16 | (sel + 5) << 24);
    dst[j * PN] = __builtin_amdgcn_perm(s[2], t, 0x0c000100u | (sel + 4) << 16);
    dst[(j + 1) * PN] = __builtin_amdgcn_perm(s[2], t, 0x0c000302u | (sel + 5) << 16);
  }
  if constexpr (M % 2 == 1) {  // the last digit alone: (c0, c1, c2 byte sel, 0)
    constexpr int j = M - 1;
    const uint32_t* s = j < 4 ? lo : hi;
    constexpr uint32_t sel = j & 3;
    const uint32_t t01 = __builtin_amdgcn_perm(s[1], s[0], 0x0c0c0400u | (sel << 8) | sel);
    dst[j * PN] = __builtin_amdgcn_perm(s[2], t01, 0x0c040100u | (sel << 16));
  }
}

// Per-element FP64 product: y = lam_s AL ue + mu_s AM ue.
template <int ELEM>
__device__ inline void element_fp64(const double ue[24], double lam_s, double mu_s, double y[24]) {
#pragma unroll
  for (int m = 0; m < 24; ++m) {
    double sl = 0.0, sm = 0.0;
#pragma unroll
    for (int n = 0; n < 24; ++n) {
      sl = fma((double)elem_al<ELEM>(m, n), ue[n], sl);
      sm = fma((double)elem_am<ELEM>(m, n), ue[n], sm);
    }
    y[m] = lam_s * sl + mu_s * sm;
  }
}

// Sum-factorised OVFEM element product, y = K_e u_e with K_e = lam_h K_lam + mu_h K_mu
// (lam_h = h lam_e, mu_h = h mu_e); the same operator as element_fp64<0>, rewritten
// without approximation.  The gradient of the octant basis (Eq. (7)) is a difference
// across a mid-plane, so every psi-weighted displacement gradient of Eq. (5) is a
// scaled Walsh coefficient of the 8 corner values: with chi_S(alpha) = prod_{k in S}
// rbar_k(alpha) and W_i[S] = sum_alpha chi_S(alpha) u_{alpha,i},
//     (psi^b, d_j u_i)_e = (1/4) (1/2)^|b| W_i[b + {j}]     (j not in b),
// b the set of axes where the stress monomial psi^b of Eq. (8) has exponent 1.  With
// (psi^b psi^b)_e = 3^-|b| (h = 1) and the isotropic stress of the symmetric gradient,
//     y_{alpha,c} = sum_S chi_S(alpha) V_c[S],
//     V_c[S] = sum over (b, j not in b, b + {j} = S) of (1/16)(3/4)^|b| s_b(c, j),
//     s_b(c, j) = lam_h tr_b delta_cj + mu_h (W_c[b + {j}] + W_j[b + {c}]),
//     tr_b = sum_{i not in b} W_i[b + {i}].
// Both transforms are 3-level butterflies: about 250 flops per element instead of the
// 2304 of the dense product.  The kernel forms W and tr once (sf_transform), then each
// output component in turn (sf_component), so that only one component's V is live.
// The lumped trilinear element (2 x 2 x 2 Gauss points, which integrate its stiffness
// exactly) has the same form: its displacement is the multilinear polynomial
// (1/8) sum_S W[S] r^S, the monomials are orthogonal with (r^T, r^T) = 8 3^-|T| on the
// reference cube, and the energy of the strain moments gives the weights
// (1/16)(1/3)^|b| in place of OVFEM's (1/16)(3/4)^|b| (ELEM = 1): the two elements differ
// only in how strongly the strain moments that vary across the element are weighted.
constexpr int kSfB[7] = {0, 1, 2, 4, 3, 6, 5};  // the seven stress monomials b as axis masks

__device__ inline void sf_transform(const double ue[24], double W[3][8], double tr[7]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int a = 0; a < 8; ++a) W[i][a] = ue[3 * a + i];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int a = 0; a < 8; ++a)
        if (!((a >> k) & 1)) {
          const double lo = W[i][a], hi = W[i][a | (1 << k)];
          W[i][a] = lo + hi;            // k not in S
          W[i][a | (1 << k)] = hi - lo;  // k in S: rbar_k = +1 at bit 1, -1 at bit 0
        }
  }
#pragma unroll
  for (int ib = 0; ib < 7; ++ib) {
    const int b = kSfB[ib];
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (!((b >> i) & 1)) t += W[i][b | (1 << i)];
    tr[ib] = t;
  }
}

// Component c of y: y[alpha] = y_{alpha,c}, alpha = 0..7.  ELEM: 0 OVFEM, 1 trilinear.
template <int ELEM>
__device__ inline void sf_component(const double W[3][8], const double tr[7], double lam_h, double mu_h, int c,
                                    double y[8]) {
  double V[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) V[a] = 0.0;
  constexpr double q = ELEM == 1 ? 1.0 / 3.0 : 0.75;  // weight ratio per axis of a strain moment
  const double f0 = 1.0 / 16.0, f1 = f0 * q, f2 = f1 * q;
  const double lb[3] = {lam_h * f0, lam_h * f1, lam_h * f2}, mb[3] = {mu_h * f0, mu_h * f1, mu_h * f2};
#pragma unroll
  for (int ib = 0; ib < 7; ++ib) {
    const int b = kSfB[ib];
    const int nb = (b & 1) + ((b >> 1) & 1) + ((b >> 2) & 1);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if ((b >> j) & 1) continue;
      const int S = b | (1 << j);
      double g = W[c][S];                            // (psi^b, d_j u_c) up to the factor
      if (!((b >> c) & 1)) g += W[j][b | (1 << c)];  // + (psi^b, d_c u_j)
      double sig = mb[nb] * g;
      if (c == j) sig = fma(lb[nb], tr[ib], sig);
      V[S] += sig;
    }
  }
#pragma unroll
  for (int k = 2; k >= 0; --k)
#pragma unroll
    for (int a = 0; a < 8; ++a)
      if (!((a >> k) & 1)) {
        const double v0 = V[a], v1 = V[a | (1 << k)];
        V[a] = v0 - v1;            // rbar_k = -1
        V[a | (1 << k)] = v0 + v1;  // rbar_k = +1
      }
#pragma unroll
  for (int a = 0; a < 8; ++a) y[a] = V[a];
}

// v of the lane one to the left within its row of 16 lanes (0 for the first lane).
__device__ inline double row_shift_right(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x111, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x111, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Values of row 1 moved to row 0 and of row 3 to row 2 (rows of 16 lanes).
__device__ inline double rows_down(double v) {
  const int lo = (int)__double2loint(v), hi = (int)__double2hiint(v);
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double((int)h[1], (int)l[1]);
}

// Magnitude key of a double: its high word with the sign cleared.  Keys order as the
// magnitudes do (not strictly), and the biased exponent b = key >> 20 bounds every
// value of a smaller or equal key: |v| < 2^(max(b, 1) - 1022).
__device__ inline uint32_t mag_key(double v) { return (uint32_t)__double2hiint(v) & 0x7fffffffu; }

__device__ inline uint32_t node_key(const D3& v) {
  return max(mag_key(v.v[0]), max(mag_key(v.v[1]), mag_key(v.v[2])));
}

// Smallest multiple S of EXP_QUANT, S >= EXP_FLOOR, with |v| < 2^S for every v whose key
// is <= key.
__device__ inline int key_exponent(uint32_t key) {
  const int e = max(max((int)(key >> 20), 1) - 1022, EXP_FLOOR);
  return (e + EXP_QUANT - 1) & ~(EXP_QUANT - 1);  // rounds up for negative e too
}

// Maximum over the wave (every lane gets it): DPP within rows of 16, then the four rows.
__device__ inline uint32_t wave_max_u32(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false));   // quad [1,0,3,2]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false));   // quad [2,3,0,1]
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false));  // row_ror 4
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false));  // row_ror 8
  const uint32_t r0 = __builtin_amdgcn_readlane((int)v, 0), r1 = __builtin_amdgcn_readlane((int)v, 16);
  const uint32_t r2 = __builtin_amdgcn_readlane((int)v, 32), r3 = __builtin_amdgcn_readlane((int)v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// One work-group tile (tile index wg of its unit) of one time step (or one matvec).
// M: digit stages of PATH_INT8 (the other paths take M = 8).  DAMP: Rayleigh-damped
// step (MODE_STEP only).
// LATE: load the owned node's u^n, u^{n-1} and dt^2/m just before its update instead of
// carrying them through the element phase (fewer live registers: the INT8 one-unit
// kernel then fits 128 VGPRs, four waves per SIMD).
// ELEM: element matrices of the FP64 path (0 OVFEM, 1 trilinear); the INT8 paths take
// theirs from the A-operand tables.
// TY: element rows of the tile (Tile<TY>).
template <int PATH, int MODE, int M, bool DAMP = false, bool LATE = false, int ELEM = 0, int TY = 16>
__device__ __forceinline__ void layer_tile(const KArgs& A, const int wg, const long long step) {
  static_assert(!DAMP || MODE == MODE_STEP, "damping applies to time steps");
  using St = Stages<M>;
  using Tl = Tile<TY>;
  constexpr int NT = Tl::THREADS, PNY = Tl::PNY;
  constexpr int IPLANE = Tl::template iplane<M>();
  constexpr int QB = PATH == PATH_INT8 ? St::QB : QBITS;
  const Geom g = A.g;
  const int tx = wg % g.tiles_x, ty = (wg / g.tiles_x) % g.tiles_y, tzc = wg / (g.tiles_x * g.tiles_y);
  const int x0 = tx * TN, y0 = ty * Tl::NY, z0 = tzc * g.tz;
  const int z1 = min(z0 + g.tz, g.nz + 1);  // owned planes [z0, z1)
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ta = t & 15, tb = t >> 4;       // element column (ta, tb); main staged node (ta+1, tb+1)

  // in-plane node sums: lsum[q] from elements of row q, usum[q-1] from elements of row q-1
  __shared__ double lsum[TY * 3 * TE];  // [q][c][p], q = 0..TY-1
  __shared__ double usum[TY * 3 * TE];  // [q-1][c][p], q = 1..TY
  __shared__ __attribute__((aligned(16))) uint32_t keys[2][Tl::WAVES];  // per wave: magnitude keys of staged planes
  constexpr bool F64 = is_f64_path(PATH);
  __shared__ __attribute__((aligned(16))) double matl[F64 ? 2 : 2 * NT];  // slices: [b][a] material
  constexpr int RING_BYTES = F64 ? 2 * Tl::FPLANE * 8 : (PATH == PATH_BF16 ? 2 * Tl::DPLANE * 4 : 2 * IPLANE * 4);
  __shared__ __attribute__((aligned(16))) unsigned char ring_raw[RING_BYTES];
  double* ringf = reinterpret_cast<double*>(ring_raw);
  uint32_t* ringd = reinterpret_cast<uint32_t*>(ring_raw);

  // INT8 staging exponent S of the current element layer (uniform over the work-group)
  int S = 0;
  v8bf a_frag[3];
  long a_frag8[3];
  if (PATH == PATH_BF16) {
#pragma unroll
    for (int i = 0; i < 3; ++i) a_frag[i] = __builtin_bit_cast(v8bf, A.alane[i * 64 + lane]);
  }
  if (PATH == PATH_INT8) {
#pragma unroll
    for (int i = 0; i < 3; ++i) a_frag8[i] = (long)A.alane8[i * 64 + lane];
  }

  // staged nodes: main node (ta+1, tb+1); the first TY + 17 lanes of the last wave stage
  // one more (the row q = 0 and the column p = 0 of the plane).  (Dealing the extra
  // nodes over all the waves measured 5 % slower: every wave then issues the extra
  // node's digit split, for a few active lanes.)
  const int xi = t - (NT - 64);
  const bool has_extra = xi >= 0 && xi < Tl::EXTRA;
  const int mp = ta + 1, mq = tb + 1;
  const int xp = xi < PN ? xi : 0, xq = xi < PN ? 0 : xi - (PN - 1);
  const NodeRef main_ref = node_ref(g, x0 - 1 + mp, y0 - 1 + mq);
  const NodeRef extra_ref = node_ref(g, x0 - 1 + xp, y0 - 1 + xq);
  const ElemRef elem = elem_ref(g, x0 - 1 + ta, y0 - 1 + tb);
  const bool owner = ta < TN && tb < Tl::NY;  // owns node (x0+ta, y0+tb) = plane (ta+1, tb+1)
  const bool owner_in = owner && main_ref.xy_ok;
  const size_t plane_bytes = (size_t)24 * (g.nx + 1) * (g.ny + 1);
  const size_t layer_bytes = (size_t)16 * g.nx * g.ny;
  const unsigned char* u_base = reinterpret_cast<const unsigned char*>(A.u);
  const unsigned char* up_base = reinterpret_cast<const unsigned char*>(A.uprev);
  const unsigned char* mat_base = reinterpret_cast<const unsigned char*>(A.mat);

  D3 u_main_next, u_extra_next = {{0.0, 0.0, 0.0}};
  D3 u_own_top = {{0.0, 0.0, 0.0}}, u_own_bot;
  double top_f[12];    // FP64: this element's contribution to the plane above
  double top_i[4][3];  // INT8: per tile row, this lane's corner contribution to the plane above
#pragma unroll
  for (int i = 0; i < 12; ++i) top_f[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) top_i[i][0] = top_i[i][1] = top_i[i][2] = 0.0;
  double2 mat_next;
  const int src_lo = A.src_ptr[wg], src_hi = A.src_ptr[wg + 1];
  const int rec_lo = A.rec_ptr[wg], rec_hi = A.rec_ptr[wg + 1];

  const int nrel = z1 - z0 + 2;  // staged planes z0-1 .. z1
  // node values of staged plane rel (rel 0 = plane z0-1): the main node, and the extra
  // node of the threads that have one (0 elsewhere)
  auto load_plane = [&](int rel, D3& m, D3& x) {
    const int Z = z0 - 1 + rel;
    const bool z_ok = Z >= 0 && Z <= g.nz;
    const unsigned char* plane = u_base + (size_t)(z_ok ? Z : 0) * plane_bytes;
    m = load_node(plane, main_ref, z_ok);
    if (has_extra) x = load_node(plane, extra_ref, z_ok);
    if constexpr (DAMP) {
      // stage w = u^n + b (u^n - u^{n-1}); the owned nodes' u^n is reloaded in the
      // node phase
      const unsigned char* pplane = up_base + (size_t)(z_ok ? Z : 0) * plane_bytes;
      const D3 pm = load_node(pplane, main_ref, z_ok);
#pragma unroll
      for (int c = 0; c < 3; ++c) m.v[c] = fma(A.damp_b, m.v[c] - pm.v[c], m.v[c]);
      if (has_extra) {
        const D3 px = load_node(pplane, extra_ref, z_ok);
#pragma unroll
        for (int c = 0; c < 3; ++c) x.v[c] = fma(A.damp_b, x.v[c] - px.v[c], x.v[c]);
      }
    }
  };
  auto fetch = [&](int rel) { load_plane(rel, u_main_next, u_extra_next); };
  auto fetch_mat = [&](int k) {
    const bool z_ok = k >= 0 && k < g.nz;
    mat_next = load_material(mat_base + (size_t)(z_ok ? k : 0) * layer_bytes, elem, z_ok);
  };
  auto stage = [&](int slot, const D3& m, const D3& x) {
    if (F64) {
      double* P = ringf + slot * Tl::FPLANE;
#pragma unroll
      for (int c = 0; c < 3; ++c) P[(c * PNY + mq) * PN + mp] = m.v[c];
      if (has_extra)
#pragma unroll
        for (int c = 0; c < 3; ++c) P[(c * PNY + xq) * PN + xp] = x.v[c];
    } else if (PATH == PATH_BF16) {
      uint32_t* P = ringd + slot * Tl::DPLANE;
      stage_digits(m, S, P + mq * DROW + 2 * mp);
      if (has_extra) stage_digits(x, S, P + xq * DROW + 2 * xp);
    } else {
      uint32_t* P = ringd + slot * IPLANE;
      stage_digits_i8<M>(m, S, P + mq * St::ROW + mp);
      if (has_extra) stage_digits_i8<M>(x, S, P + xq * St::ROW + xp);
    }
  };
  // work-group maximum of the keys written by the four waves into keys[slot]
  auto read_keys = [&](int slot) -> uint32_t {
    uint32_t k = 0;
#pragma unroll
    for (int w4 = 0; w4 < Tl::WAVES; w4 += 4) {
      const uint4 k4 = *reinterpret_cast<const uint4*>(keys[slot] + w4);
      k = max(k, max(max(k4.x, k4.y), max(k4.z, k4.w)));
    }
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
  };

  // Staging exponent (INT8).  Layer it (planes rel it, it+1) needs every staged value
  // below 2^S; S(it) = key_exponent of the larger key of the two planes.  key_top: the
  // key of plane it+1 while layer it runs.
  uint32_t key_top = 0;
  bool restage = false;  // plane it (already staged for layer it-1) must be staged again
  if (F64) {
    fetch(0);
    stage(0, u_main_next, u_extra_next);
    fetch(1);
  } else {
    D3 m0, x0 = {{0.0, 0.0, 0.0}};
    load_plane(0, m0, x0);
    fetch(1);
    const uint32_t k0 = wave_max_u32(max(node_key(m0), node_key(x0)));
    const uint32_t k1 = wave_max_u32(max(node_key(u_main_next), node_key(u_extra_next)));
    if (lane == 0) {
      keys[0][wave] = k0;
      keys[1][wave] = k1;
    }
    __syncthreads();
    const uint32_t K0 = read_keys(0);
    key_top = read_keys(1);
    S = key_exponent(max(K0, key_top));
    stage(0, m0, x0);
  }
  fetch_mat(z0 - 1);

  for (int it = 0; it + 1 < nrel; ++it) {
    const int k = z0 - 1 + it;  // element layer: planes rel it (slot it&1) and it+1
    const int bot = it & 1, top = (it + 1) & 1;
    u_own_bot = u_own_top;
    u_own_top = u_main_next;
    if (!F64 && restage) {
      D3 rm, rx = {{0.0, 0.0, 0.0}};
      load_plane(it, rm, rx);
      stage(bot, rm, rx);
    }
    stage(top, u_main_next, u_extra_next);
    const double2 mat_e = mat_next;
    if (!F64) {
      matl[2 * t] = mat_e.x;
      matl[2 * t + 1] = mat_e.y;
    }
    if (it + 2 < nrel) {
      fetch(it + 2);
      fetch_mat(k + 1);
    }
    const bool do_node = it >= 1 && owner_in;
    const size_t node_off = (size_t)k * plane_bytes + main_ref.off;  // byte offset of owned node
    double up[3] = {0.0, 0.0, 0.0}, ac = 0.0;
    auto load_node_state = [&]() {
      if (do_node && MODE == MODE_STEP) {
        const double* pp =
            reinterpret_cast<const double*>(reinterpret_cast<const unsigned char*>(A.uprev) + node_off);
        up[0] = pp[0];
        up[1] = pp[1];
        up[2] = pp[2];
        if constexpr (DAMP || LATE) {
          const double* pu = reinterpret_cast<const double*>(u_base + node_off);
          u_own_bot.v[0] = pu[0];
          u_own_bot.v[1] = pu[1];
          u_own_bot.v[2] = pu[2];
        }
        ac = *reinterpret_cast<const double*>(reinterpret_cast<const unsigned char*>(A.acoef) +
                                              (size_t)k * (plane_bytes / 3) + main_ref.off / 3);
      }
    };
    if constexpr (!LATE) load_node_state();
    const bool layer_ok = k >= 0 && k < g.nz;
    __syncthreads();

    // ---- element layer k -> in-plane sums for plane k
    if (F64) {
      // bottom-corner contributions (with the previous layer's top ones) go to the in-plane
      // sums of plane k; top-corner contributions are kept for plane k + 1
      double y[24];
      if (layer_ok) {
        const double* Pb = ringf + bot * Tl::FPLANE;
        const double* Pt = ringf + top * Tl::FPLANE;
        double ue[24];
#pragma unroll
        for (int alpha = 0; alpha < 8; ++alpha) {
          const int di = alpha & 1, dj = (alpha >> 1) & 1, dk = alpha >> 2;
          const double* P = dk ? Pt : Pb;
#pragma unroll
          for (int c = 0; c < 3; ++c) ue[3 * alpha + c] = P[(c * PNY + tb + dj) * PN + ta + di];
        }
        if constexpr (PATH == PATH_FP64SF) {
          // one output component at a time (fewer live registers)
          double W[3][8], tr[7];
          sf_transform(ue, W, tr);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double yc[8];
            // mat holds h lam / kElemScaleLam, h mu / kElemScaleMu
            sf_component<ELEM>(W, tr, mat_e.x * kElemScaleLam[ELEM], mat_e.y * kElemScaleMu[ELEM], c, yc);
            const double v0 = yc[0] + top_f[c], v1 = yc[1] + top_f[3 + c];
            const double v2 = yc[2] + top_f[6 + c], v3 = yc[3] + top_f[9 + c];
            lsum[(tb * 3 + c) * TE + ta] = v0 + row_shift_right(v1);  // node (ta, tb)
            usum[(tb * 3 + c) * TE + ta] = v2 + row_shift_right(v3);  // node (ta, tb + 1)
#pragma unroll
            for (int a = 0; a < 4; ++a) top_f[3 * a + c] = yc[4 + a];
          }
        } else {
          element_fp64<ELEM>(ue, mat_e.x, mat_e.y, y);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 24; ++i) y[i] = 0.0;
      }
      if (PATH != PATH_FP64SF || !layer_ok) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double v0 = y[c] + top_f[c], v1 = y[3 + c] + top_f[3 + c];
          const double v2 = y[6 + c] + top_f[6 + c], v3 = y[9 + c] + top_f[9 + c];
          lsum[(tb * 3 + c) * TE + ta] = v0 + row_shift_right(v1);  // node (ta, tb)
          usum[(tb * 3 + c) * TE + ta] = v2 + row_shift_right(v3);  // node (ta, tb + 1)
        }
#pragma unroll
        for (int i = 0; i < 12; ++i) top_f[i] = y[12 + i];
      }
    } else {
      const int ja = lane & 15, G = lane >> 4;  // element column; lane group
      const uint32_t* Pin = ringd + ((G >> 1) ? top : bot) * (PATH == PATH_BF16 ? Tl::DPLANE : IPLANE);
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        const int b = 4 * wave + tt;
        double ybot[3] = {0.0, 0.0, 0.0}, ytop[3] = {0.0, 0.0, 0.0};
        if (layer_ok) {
          const double2 me = *reinterpret_cast<const double2*>(matl + 2 * (b * TE + ja));
          double R[12];
          constexpr int NGRP = PATH == PATH_INT8 ? St::NG : NPAIR;
#pragma unroll
          for (int p = NGRP - 1; p >= 0; --p) {
            if constexpr (PATH == PATH_BF16) {
              // the lane's eight K slots: (c0, c1, c2, 0) of node ja, then of node ja+1
              const uint32_t* P = Pin + (b + (G & 1)) * DROW + 2 * ja;
              const uint2* ph = reinterpret_cast<const uint2*>(P + (2 * p) * PN * 2);
              const uint2* pl = reinterpret_cast<const uint2*>(P + (2 * p + 1) * PN * 2);
              const uint2 h0 = ph[0], h1 = ph[1], l0 = pl[0], l1 = pl[1];
              const v4u bh = {h0.x, h0.y, h1.x, h1.y};
              const v4u bl = {l0.x, l0.y, l1.x, l1.y};
              const v8bf Bh = __builtin_bit_cast(v8bf, bh), Bl = __builtin_bit_cast(v8bf, bl);
              const v4f z = {0.0f, 0.0f, 0.0f, 0.0f};
              v4f c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag[0], Bh, z, 0, 0, 0);
              v4f c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag[1], Bh, z, 0, 0, 0);
              v4f c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag[2], Bh, z, 0, 0, 0);
              c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag[0], Bl, c0, 0, 0, 0);
              c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag[1], Bl, c1, 0, 0, 0);
              c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_frag[2], Bl, c2, 0, 0, 0);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                if (p == NGRP - 1) {
                  R[r] = (double)c0[r];
                  R[4 + r] = (double)c1[r];
                  R[8 + r] = (double)c2[r];
                } else {
                  R[r] = fma(R[r], 65536.0, (double)c0[r]);
                  R[4 + r] = fma(R[4 + r], 65536.0, (double)c1[r]);
                  R[8 + r] = fma(R[8 + r], 65536.0, (double)c2[r]);
                }
              }
            } else {
              // digit words of node ja and ja+1 for digits 2p+1 (hi, absent in the top
              // group when M is odd) and 2p (lo)
              const uint32_t* P = Pin + (b + (G & 1)) * St::ROW + ja;
              const long Bl = (long)((uint64_t)P[(2 * p) * PN] | ((uint64_t)P[(2 * p) * PN + 1] << 32));
              const v4i z = {0, 0, 0, 0};
              v4i c0 = z, c1 = z, c2 = z;
              if (2 * p + 1 < M) {
                const long Bh =
                    (long)((uint64_t)P[(2 * p + 1) * PN] | ((uint64_t)P[(2 * p + 1) * PN + 1] << 32));
                c0 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_frag8[0], Bh, z, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_frag8[1], Bh, z, 0, 0, 0);
                c2 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_frag8[2], Bh, z, 0, 0, 0);
                c0 = c0 << 8;
                c1 = c1 << 8;
                c2 = c2 << 8;
              }
              c0 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_frag8[0], Bl, c0, 0, 0, 0);
              c1 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_frag8[1], Bl, c1, 0, 0, 0);
              c2 = __builtin_amdgcn_mfma_i32_16x16x32_i8(a_frag8[2], Bl, c2, 0, 0, 0);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                if (p == NGRP - 1) {
                  R[r] = (double)c0[r];
                  R[4 + r] = (double)c1[r];
                  R[8 + r] = (double)c2[r];
                } else {
                  R[r] = fma(R[r], 65536.0, (double)c0[r]);
                  R[4 + r] = fma(R[4 + r], 65536.0, (double)c1[r]);
                  R[8 + r] = fma(R[8 + r], 65536.0, (double)c2[r]);
                }
              }
            }
          }
          // output s = 4 * row tile + reg: s < 6 rows of AL, s >= 6 rows of AM;
          // dk = (s % 6) / 3, c = s % 3, at corner G + 4 dk
          const double sl = ldexp(me.x, S - QB), sm = ldexp(me.y, S - QB);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            ybot[c] = R[c] * sl + R[6 + c] * sm;
            ytop[c] = R[3 + c] * sl + R[9 + c] * sm;
          }
        }
        // lane (ja, G) holds corner G of element (ja, b): node (ja + (G & 1), b + (G >> 1)).
        // Each in-plane node of the row gets two terms: the even lanes store, then the
        // odd lanes add (LDS operations of one wave complete in order; two addends
        // commute exactly, so the sum does not depend on the hardware's lane order).
        double v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          v[c] = ybot[c] + top_i[tt][c];
          top_i[tt][c] = ytop[c];
        }
        double* dst = (G >> 1 ? usum : lsum) + b * 3 * TE + ja + (G & 1);
        if ((G & 1) == 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) dst[c * TE] = v[c];
        }
        if ((G & 1) == 1 && ja < TE - 1) {
#pragma unroll
          for (int c = 0; c < 3; ++c) __hip_atomic_fetch_add(dst + c * TE, v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __builtin_amdgcn_sched_barrier(0);  // keep tile rows apart: bounds live registers
      }
      // key of the plane fetched for the next layer (its loads had the element phase to land)
      if (it + 2 < nrel) {
        const uint32_t kk = wave_max_u32(max(node_key(u_main_next), node_key(u_extra_next)));
        if (lane == 0) keys[0][wave] = kk;
      }
    }
    __syncthreads();

    if (!F64 && it + 2 < nrel) {
      // exponent of the next layer (planes it+1, it+2); a change restages plane it+1
      // (its values are reloaded when the next layer starts)
      const uint32_t key_new = read_keys(0);
      const int L = key_exponent(max(key_top, key_new));
      key_top = key_new;
      restage = L != S;
      S = L;
    }

    // ---- node phase for plane Z = k (owned when it >= 1)
    if constexpr (LATE) load_node_state();
    if (do_node) {
      const int p = ta + 1, q = tb + 1;
      double f[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) f[c] = lsum[(q * 3 + c) * TE + p] + usum[((q - 1) * 3 + c) * TE + p];
      const long long nid = (long long)k * (g.nx + 1) * (g.ny + 1) + main_ref.off / 24;
      if (MODE == MODE_MATVEC) {
        double* o = A.ku + 3 * nid;
        o[0] = f[0];
        o[1] = f[1];
        o[2] = f[2];
      } else {
        double F[3] = {0.0, 0.0, 0.0};
        for (int s = src_lo; s < src_hi; ++s)
          if (A.src_node[s] == (int)nid && step < A.src_nt) {
            const double w = A.wavelet[(long long)A.src_row[s] * A.src_nt + step];
            const int sc = A.src_comp[s];
            F[0] += sc == 0 ? w : 0.0;
            F[1] += sc == 1 ? w : 0.0;
            F[2] += sc == 2 ? w : 0.0;
          }
        double un[3];
        if constexpr (DAMP) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            un[c] = ac > 0.0 ? A.damp_c1 * u_own_bot.v[c] - A.damp_c2 * up[c] + ac * (F[c] - f[c]) : 0.0;
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c)
            un[c] = ac > 0.0 ? 2.0 * u_own_bot.v[c] - up[c] + ac * (F[c] - f[c]) : 0.0;
        }
        double* o = A.unext + 3 * nid;
        o[0] = un[0];
        o[1] = un[1];
        o[2] = un[2];
        for (int r = rec_lo; r < rec_hi; ++r)
          if (A.rec_node[r] == (int)nid && step < A.rec_nt) {
            double* tr = A.traces + (long long)A.rec_idx[r] * 3 * A.rec_nt + step;
            tr[0] = un[0];
            tr[A.rec_nt] = un[1];
            tr[2 * A.rec_nt] = un[2];
          }
      }
    }
  }
}

// The shots of one grid (A.n_units of them, laid out at fixed strides): one work-group
// per tile and shot, work items remapped so each XCD takes a contiguous run.  The step
// index is *step_base + step (step_base may be null), so a captured sequence of launches
// can be replayed with a step base kept in device memory.  The i8 kernels are held to
// four waves per SIMD (128 registers): the damped and the 6-digit forms otherwise take
// 129-131 and drop to three, which costs them 8-9 %.
template <int PATH, int MODE, int M = 8, bool DAMP = false, int ELEM = 0, int TY = 16>
__global__ void __launch_bounds__(Tile<TY>::THREADS, groups_per_cu(PATH, TY))
    ovfem_layer_kernel(KArgs A, const long long* step_base, long long step) {
  const long long s = (step_base ? *step_base : 0) + step;
  const int units = A.n_units > 1 ? A.n_units : 1;
  const int item = logical_tile(blockIdx.x, A.g.n_wg * units);
  const int v = item / A.g.n_wg;
  if (v > 0) {
    A.u += v * A.unit_u;
    A.uprev += v * A.unit_u;
    A.unext += v * A.unit_u;
    A.src_ptr += v * A.unit_src;
    A.traces += v * A.unit_tr;
  }
  layer_tile<PATH, MODE, M, DAMP, PATH == PATH_INT8, ELEM, TY>(A, item - v * A.g.n_wg, s);
}

// Many units in one launch (grids of uneven size, each with its shots): unit u owns work
// items [unit_begin[u], unit_begin[u+1]) and is found by binary search; its own step
// offset is units[u].step.  Work items are remapped so that each XCD gets a contiguous
// run.  ovfem_batch_kernel takes one work item per work-group;
// ovfem_batch_strided_kernel runs on a grid smaller than the work list and strides over
// it (the grid size is then a multiple of 8, so a work-group stays on one XCD's run).
// Unit v's argument record, read field by field through the constant address space:
// the records are written by the host before the launch and never by a kernel, and
// invariant loads let the compiler treat the fields as it treats kernel arguments (the
// i8 batch kernel then fits in 128 registers instead of 144).
__device__ inline KArgs load_unit(const KArgs* units, int v) {
  static_assert(sizeof(KArgs) == 248, "load_unit copies every field of KArgs: keep the two in step");
  using CK = const __attribute__((address_space(4))) KArgs;
  CK* p = reinterpret_cast<CK*>(reinterpret_cast<uintptr_t>(units)) + v;
  KArgs a;
  a.g.nx = p->g.nx;
  a.g.ny = p->g.ny;
  a.g.nz = p->g.nz;
  a.g.tz = p->g.tz;
  a.g.tiles_x = p->g.tiles_x;
  a.g.tiles_y = p->g.tiles_y;
  a.g.chunks = p->g.chunks;
  a.g.n_wg = p->g.n_wg;
  a.g.ty = p->g.ty;
  a.u = p->u;
  a.uprev = p->uprev;
  a.unext = p->unext;
  a.ku = p->ku;
  a.mat = p->mat;
  a.acoef = p->acoef;
  a.alane = p->alane;
  a.alane8 = p->alane8;
  a.src_ptr = p->src_ptr;
  a.src_node = p->src_node;
  a.src_comp = p->src_comp;
  a.src_row = p->src_row;
  a.wavelet = p->wavelet;
  a.rec_ptr = p->rec_ptr;
  a.rec_node = p->rec_node;
  a.rec_idx = p->rec_idx;
  a.traces = p->traces;
  a.src_nt = p->src_nt;
  a.rec_nt = p->rec_nt;
  a.step = p->step;
  a.damp_b = p->damp_b;
  a.damp_c1 = p->damp_c1;
  a.damp_c2 = p->damp_c2;
  a.n_units = p->n_units;
  a.unit_u = p->unit_u;
  a.unit_src = p->unit_src;
  a.unit_tr = p->unit_tr;
  return a;
}

__device__ inline int find_unit(const int* unit_begin, int n_units, int item) {
  int lo = 0, hi = n_units - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (unit_begin[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int PATH, int MODE, int M = 8, bool DAMP = false, int ELEM = 0, int TY = 16>
__global__ void __launch_bounds__(Tile<TY>::THREADS, groups_per_cu(PATH, TY))
    ovfem_batch_kernel(const KArgs* units, const int* unit_begin, int n_units, int total,
                       const long long* step_base, long long step) {
  const long long s = (step_base ? *step_base : 0) + step;
  const int item = logical_tile(blockIdx.x, total);
  const int v = find_unit(unit_begin, n_units, item);
  const KArgs A = load_unit(units, v);
  layer_tile<PATH, MODE, M, DAMP, PATH == PATH_INT8, ELEM, TY>(A, item - unit_begin[v], s + A.step);
}

template <int PATH, int MODE, int M = 8, bool DAMP = false, int ELEM = 0, int TY = 16>
__global__ void __launch_bounds__(Tile<TY>::THREADS, is_f64_path(PATH) || TY == 32 ? 1 : 2)
    ovfem_batch_strided_kernel(const KArgs* units, const int* unit_begin, int n_units, int total,
                               const long long* step_base, long long step) {
  const long long s = (step_base ? *step_base : 0) + step;
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    const int item = logical_tile(b, total);
    const int v = find_unit(unit_begin, n_units, item);
    const KArgs A = load_unit(units, v);
    layer_tile<PATH, MODE, M, DAMP, false, ELEM, TY>(A, item - unit_begin[v], s + A.step);
    __syncthreads();  // LDS is reused by the next work item
  }
}

// Adds n to the device step base (last node of a captured block of steps).
static __global__ void ovfem_advance_step_kernel(long long* step_base, long long n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_base += n;
}

}  // namespace ovfem
