// Integer reference matrices of the voxel elements, derived at compile time: the OVFEM
// element (below) and the trilinear comparison element (further down).
//
// Sec. 2, Eq. (5): K_e = (psi grad phi)^T (psi psi)^{-1} c (psi grad phi), with the
// octant-indicator displacement basis of Eq. (7) and the seven stress monomials of
// Eq. (8) used for every stress component.  For an isotropic c = lam C_lam + mu C_mu
// (Voigt, engineering shear) the element matrix is K_e = h (lam K_lam + mu K_mu).
// This header evaluates the element integrals in exact rationals and returns
//     AL = 256 K_lam  and  AM = 128 K_mu,
// which are integer matrices with entries inside the INT8 range (the paper's
// K^INT8 of Eq. (9) is the equivalent kappa/G form); the compile-time checks below
// fail the build if either is not integral or does not fit.
//
// Local node alpha = di + 2 dj + 4 dk sits at rbar = (2di-1, 2dj-1, 2dk-1); element
// DOF index 3 alpha + c.  Lengths are in units of h (the matrices are for h = 1).
#pragma once

namespace ovfem {

struct Rat {
  long long n, d;
};

constexpr long long gcd_ll(long long a, long long b) {
  if (a < 0) a = -a;
  if (b < 0) b = -b;
  while (b) {
    long long t = a % b;
    a = b;
    b = t;
  }
  return a;
}
constexpr Rat rat(long long n, long long d) {
  if (d < 0) {
    n = -n;
    d = -d;
  }
  long long g = gcd_ll(n, d);
  if (g == 0) g = 1;
  return Rat{n / g, d / g};
}
constexpr Rat rmul(Rat a, Rat b) { return rat(a.n * b.n, a.d * b.d); }
constexpr Rat radd(Rat a, Rat b) { return rat(a.n * b.d + b.n * a.d, a.d * b.d); }

// exponents (a1, a2, a3) of the stress monomials 1, r1, r2, r3, r1 r2, r2 r3, r1 r3
constexpr int kPsiExp[7][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                               {1, 1, 0}, {0, 1, 1}, {1, 0, 1}};
// Voigt rows 11, 22, 33, 23, 13, 12 as component pairs
constexpr int kVoigt[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
// C_mu = diag(2, 2, 2, 1, 1, 1); C_lam = 1 1^T on the normal block
constexpr int kCmu[6] = {2, 2, 2, 1, 1, 1};

constexpr int corner_sign(int alpha, int axis) { return 2 * ((alpha >> axis) & 1) - 1; }

// int_{-1}^{1} r^n dr
constexpr Rat integral_monomial(int n) { return (n % 2) ? Rat{0, 1} : rat(2, n + 1); }
// int_{-1}^{1} H(s r) r^a dr = int_0^1 (s t)^a dt = s^a / (a + 1)
constexpr Rat integral_half(int s, int a) { return rat((a % 2) ? s : 1, a + 1); }

// (psi^b psi^b')_e for h = 1: (1/2)^3 prod_k int r^(a_k + a'_k)
constexpr Rat psi_gram(int b, int bp) {
  Rat v = rat(1, 8);
  for (int k = 0; k < 3; ++k) v = rmul(v, integral_monomial(kPsiExp[b][k] + kPsiExp[bp][k]));
  return v;
}

// (psi^b d phi^alpha / d x_j)_e for h = 1.  d/dx_j of the octant indicator is
// 2 rbar_j delta(r_j) prod_{k != j} H(rbar_k r_k); with the (1/2)^3 volume factor
// the integral is (1/4) rbar_j psi^b|_{r_j=0} integrated over the octant face.
constexpr Rat psi_grad_phi(int j, int b, int alpha) {
  if (kPsiExp[b][j] != 0) return Rat{0, 1};
  Rat v = rat(corner_sign(alpha, j), 4);
  for (int k = 0; k < 3; ++k)
    if (k != j) v = rmul(v, integral_half(corner_sign(alpha, k), kPsiExp[b][k]));
  return v;
}

// coefficient of element DOF `dof` in the psi^b-weighted Voigt strain v
constexpr Rat strain_coef(int b, int v, int dof) {
  const int alpha = dof / 3, c = dof % 3;
  const int p = kVoigt[v][0], q = kVoigt[v][1];
  if (p == q) return c == p ? psi_grad_phi(p, b, alpha) : Rat{0, 1};
  if (c == p) return psi_grad_phi(q, b, alpha);
  if (c == q) return psi_grad_phi(p, b, alpha);
  return Rat{0, 1};
}

struct RefMats {
  int AL[24][24];  // 256 K_lam
  int AM[24][24];  // 128 K_mu
  bool ok;         // integral, in INT8 range, Gram matrix diagonal
};

constexpr RefMats make_refmats() {
  RefMats R{};
  R.ok = true;
  // the stress monomials are orthogonal on the voxel, so (psi psi)^{-1} is diagonal
  for (int b = 0; b < 7; ++b)
    for (int bp = 0; bp < 7; ++bp)
      if (b != bp && psi_gram(b, bp).n != 0) R.ok = false;
  for (int m = 0; m < 24; ++m) {
    for (int n = 0; n < 24; ++n) {
      Rat kl{0, 1}, km{0, 1};
      for (int b = 0; b < 7; ++b) {
        const Rat g = psi_gram(b, b);
        const Rat w = rat(g.d, g.n);  // 1 / (psi^b psi^b)_e
        Rat dm{0, 1}, dn{0, 1};       // psi^b-weighted volumetric strain rows
        for (int v = 0; v < 3; ++v) {
          dm = radd(dm, strain_coef(b, v, m));
          dn = radd(dn, strain_coef(b, v, n));
        }
        kl = radd(kl, rmul(w, rmul(dm, dn)));
        for (int v = 0; v < 6; ++v)
          km = radd(km, rmul(rmul(w, rat(kCmu[v], 1)), rmul(strain_coef(b, v, m), strain_coef(b, v, n))));
      }
      const Rat al = rmul(kl, rat(256, 1)), am = rmul(km, rat(128, 1));
      if (al.d != 1 || am.d != 1) R.ok = false;
      if (al.n < -128 || al.n > 127 || am.n < -128 || am.n > 127) R.ok = false;
      R.AL[m][n] = static_cast<int>(al.n);
      R.AM[m][n] = static_cast<int>(am.n);
    }
  }
  return R;
}

inline constexpr RefMats kRef = make_refmats();
static_assert(kRef.ok, "OVFEM reference matrices must be integral INT8 after scaling by 256 / 128");

// The conventional trilinear voxel element ("VFEM", the comparison element of Sec. 3):
// N_a = (1/8) prod_k (1 + s_ak r_k) with the Galerkin stiffness integrated exactly (the
// "8-point integration" is exact for it).  With G_ij(a, b) = int dN_a/dx_i dN_b/dx_j
// over the unit voxel (d/dx = 2 d/dr, dx = dr / 8):
//   G_ii(a, b) = (1/64) s_ai s_bi prod_{k != i} int (1 + s_ak r)(1 + s_bk r) dr,
//   G_ij(a, b) = (1/64) s_ai s_bj * 4 * int (1 + s_al r)(1 + s_bl r) dr (l the third axis),
// with int_{-1}^{1} (1 + s r)(1 + t r) dr = 2 + (2/3) s t; then
//   K_lam[3a+c][3b+d] = G_cd(a, b),  K_mu[3a+c][3b+d] = delta_cd sum_k G_kk(a, b) + G_dc(a, b),
// and AL = 72 K_lam, AM = 72 K_mu are integer matrices (checked below).
constexpr Rat lin_pair_integral(int s, int t) { return radd(rat(2, 1), rat(2 * s * t, 3)); }

constexpr Rat trilinear_g(int a, int b, int i, int j) {
  Rat v = rat(corner_sign(a, i) * corner_sign(b, j), 64);
  if (i == j) {
    v = rmul(v, rat(2, 1));
    for (int k = 0; k < 3; ++k)
      if (k != i) v = rmul(v, lin_pair_integral(corner_sign(a, k), corner_sign(b, k)));
  } else {
    const int l = 3 - i - j;
    v = rmul(v, rmul(rat(4, 1), lin_pair_integral(corner_sign(a, l), corner_sign(b, l))));
  }
  return rmul(v, rat(1, 2));  // r-space to x-space for h = 1: (2)^2 (1/2)^3
}

struct ElemMats {
  int AL[24][24];
  int AM[24][24];
  int scale_lam, scale_mu;  // AL = scale_lam K_lam, AM = scale_mu K_mu
  bool ok;
};

constexpr ElemMats make_trilinear() {
  ElemMats R{};
  R.ok = true;
  R.scale_lam = 72;
  R.scale_mu = 72;
  for (int m = 0; m < 24; ++m)
    for (int n = 0; n < 24; ++n) {
      const int a = m / 3, c = m % 3, b = n / 3, d = n % 3;
      Rat kl = trilinear_g(a, b, c, d);
      Rat km = trilinear_g(a, b, d, c);
      if (c == d)
        for (int k = 0; k < 3; ++k) km = radd(km, trilinear_g(a, b, k, k));
      const Rat al = rmul(kl, rat(72, 1)), am = rmul(km, rat(72, 1));
      if (al.d != 1 || am.d != 1) R.ok = false;
      if (al.n < -128 || al.n > 127 || am.n < -128 || am.n > 127) R.ok = false;
      R.AL[m][n] = static_cast<int>(al.n);
      R.AM[m][n] = static_cast<int>(am.n);
    }
  return R;
}

inline constexpr ElemMats kTri = make_trilinear();
static_assert(kTri.ok, "trilinear reference matrices must be integral INT8 after scaling by 72");

// The element types: 0 = OVFEM, 1 = trilinear.
constexpr int kElemScaleLam[2] = {256, 72};
constexpr int kElemScaleMu[2] = {128, 72};
template <int ELEM>
constexpr int elem_al(int m, int n) { return ELEM == 0 ? kRef.AL[m][n] : kTri.AL[m][n]; }
template <int ELEM>
constexpr int elem_am(int m, int n) { return ELEM == 0 ? kRef.AM[m][n] : kTri.AM[m][n]; }

// Largest row sum of |AL| and |AM|: bounds a single INT8 product stage.
constexpr int max_row_abs(const int (&A)[24][24]) {
  int best = 0;
  for (int m = 0; m < 24; ++m) {
    int s = 0;
    for (int n = 0; n < 24; ++n) s += A[m][n] < 0 ? -A[m][n] : A[m][n];
    best = s > best ? s : best;
  }
  return best;
}
constexpr int max4(int a, int b, int c, int d) {
  const int x = a > b ? a : b, y = c > d ? c : d;
  return x > y ? x : y;
}
inline constexpr int kMaxRowAbs =
    max4(max_row_abs(kRef.AL), max_row_abs(kRef.AM), max_row_abs(kTri.AL), max_row_abs(kTri.AM));

}  // namespace ovfem
