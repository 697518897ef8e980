"""Exact element matrices of the voxel elements (oracle; test infrastructure only).

OVFEM element (Sec. 2, Eqs. (4)-(8)).  A voxel of edge h is mapped to local
coordinates r in [-1, 1]^3 by x = x0 + (h/2)(r + 1).  Local node alpha = i + 2j + 4k
(i, j, k in {0, 1}) sits at rbar^alpha = (2i-1, 2j-1, 2k-1).  The displacement basis
is the octant indicator phi^alpha = H(rbar1 r1) H(rbar2 r2) H(rbar3 r3) (Eq. (7)); the
stress basis is psi = {1, r1, r2, r3, r1 r2, r2 r3, r1 r3} (Eq. (8)), used for each of
the six stress components.  Stationarity of the Hellinger-Reissner functional
(Eq. (4)) gives the element stiffness of Eq. (5),

    K_e = (psi grad phi)_e^T  (psi psi)_e^{-1}  c  (psi grad phi)_e,

and the element mass of Eq. (6), rho (phi phi)_e, which is diagonal.

Everything below is evaluated in exact rational arithmetic (fractions.Fraction):

* (psi^b psi^b')_e = (h/2)^3 prod_k int_{-1}^{1} r^(a_k + a'_k) dr.
* d phi^alpha / d x_j = (2/h) rbar_j delta(r_j) prod_{k != j} H(rbar_k r_k): the
  gradient of the octant indicator is a surface delta on the mid-plane r_j = 0, so
  (psi^b d_j phi^alpha)_e = (h/2)^2 rbar_j [psi^b restricted to r_j = 0]
  prod_{k != j} int_{-1}^{1} H(rbar_k r) r^(a_k) dr.
* Strains use Voigt order (11, 22, 33, 23, 13, 12) with engineering shear, and the
  isotropic Voigt stiffness c = lam * C_lam + mu * C_mu with C_lam = 1 1^T on the
  normal block and C_mu = diag(2, 2, 2, 1, 1, 1).

Because K_e is linear in c and scales as h, K_e = h (lam_e K_lam + mu_e K_mu) with K_lam
and K_mu the h = 1 matrices for unit lam and unit mu.  DOF index within an element is
3 * alpha + component.

Trilinear element (the conventional voxel element of Sec. 2, "VFEM").  The printed
basis carries a sign/shift typo; the standard trilinear basis
(1/8) prod (1 + rbar_i r_i) is used, integrated with 2x2x2 Gauss points (the
"8-point integration" mentioned in Sec. 3), with the lumped mass rho h^3 / 8 per
node.  It serves the dispersion comparison and, as the comparison element of Sec. 3,
the element option of the stepper.
"""
from fractions import Fraction
import itertools

import numpy as np

# exponent vectors of the stress basis psi = {1, r1, r2, r3, r1 r2, r2 r3, r1 r3}
PSI_EXPONENTS = ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
                 (1, 1, 0), (0, 1, 1), (1, 0, 1))

# Voigt strain rows: (normal component) or (pair) with engineering shear
VOIGT = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))


def node_rbar(alpha):
    """Local corner signs rbar^alpha for alpha = i + 2j + 4k."""
    i, j, k = alpha & 1, (alpha >> 1) & 1, (alpha >> 2) & 1
    return (2 * i - 1, 2 * j - 1, 2 * k - 1)


def _int_monomial(n):
    """int_{-1}^{1} r^n dr, exact."""
    return Fraction(2, n + 1) if n % 2 == 0 else Fraction(0)


def _int_heaviside_monomial(s, a):
    """int_{-1}^{1} H(s r) r^a dr for s = +-1, exact: the half interval on the side s."""
    # r = s t, t in [0, 1]:  int_0^1 (s t)^a dt = s^a / (a + 1)
    return Fraction(s ** a, a + 1)


def psi_gram(h=Fraction(1)):
    """(psi^b psi^b')_e, a 7 x 7 matrix of Fractions (Eq. (5), middle factor)."""
    h = Fraction(h)
    vol = (h / 2) ** 3
    P = [[Fraction(0)] * 7 for _ in range(7)]
    for b, ab in enumerate(PSI_EXPONENTS):
        for bp, abp in enumerate(PSI_EXPONENTS):
            v = vol
            for k in range(3):
                v *= _int_monomial(ab[k] + abp[k])
            P[b][bp] = v
    return P


def psi_grad_phi(h=Fraction(1)):
    """G[j][b][alpha] = (psi^b d phi^alpha / d x_j)_e, exact (Eq. (5), outer factors)."""
    h = Fraction(h)
    G = [[[Fraction(0)] * 8 for _ in range(7)] for _ in range(3)]
    for j in range(3):
        for b, ab in enumerate(PSI_EXPONENTS):
            if ab[j] != 0:
                continue  # psi^b vanishes on the mid-plane r_j = 0
            for alpha in range(8):
                rb = node_rbar(alpha)
                # (h/2)^3 jacobian times (2/h) from d/dx_j = (2/h) d/dr_j
                v = (h / 2) ** 2 * rb[j]
                for k in range(3):
                    if k != j:
                        v *= _int_heaviside_monomial(rb[k], ab[k])
                G[j][b][alpha] = v
    return G


def strain_operator(h=Fraction(1)):
    """Bhat[(b, v)][(alpha, c)]: coefficient of the Voigt strain v weighted by psi^b.

    42 x 24 list of Fractions; row index 6 * b + v, column 3 * alpha + c.
    """
    G = psi_grad_phi(h)
    B = [[Fraction(0)] * 24 for _ in range(42)]
    for b in range(7):
        for v, (p, q) in enumerate(VOIGT):
            row = 6 * b + v
            for alpha in range(8):
                if p == q:
                    B[row][3 * alpha + p] += G[p][b][alpha]
                else:
                    # engineering shear: d u_p / d x_q + d u_q / d x_p
                    B[row][3 * alpha + p] += G[q][b][alpha]
                    B[row][3 * alpha + q] += G[p][b][alpha]
    return B


def voigt_stiffness(lam, mu):
    """Isotropic Voigt stiffness (Fractions or floats): lam 1 1^T (normal block) + mu diag(2,2,2,1,1,1)."""
    C = [[0 * lam] * 6 for _ in range(6)]
    for a in range(3):
        for b in range(3):
            C[a][b] = C[a][b] + lam
        C[a][a] = C[a][a] + 2 * mu
    for a in range(3, 6):
        C[a][a] = C[a][a] + mu
    return C


def _frac_inverse(A):
    """Gauss-Jordan inverse of a square matrix of Fractions."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [x / pv for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [row[n:] for row in M]


def ovfem_stiffness_exact(lam, mu, h=Fraction(1)):
    """K_e of Eq. (5) for one voxel, exact: 24 x 24 list of Fractions."""
    B = strain_operator(h)
    Pinv = _frac_inverse(psi_gram(h))
    C = voigt_stiffness(Fraction(lam), Fraction(mu))
    K = [[Fraction(0)] * 24 for _ in range(24)]
    for b in range(7):
        for bp in range(7):
            w = Pinv[b][bp]
            if w == 0:
                continue
            for v in range(6):
                for vp in range(6):
                    cw = w * C[v][vp]
                    if cw == 0:
                        continue
                    rb, rbp = B[6 * b + v], B[6 * bp + vp]
                    for m in range(24):
                        if rb[m] == 0:
                            continue
                        f = rb[m] * cw
                        for n in range(24):
                            if rbp[n] != 0:
                                K[m][n] += f * rbp[n]
    return K


_CACHE = {}


def ovfem_reference_exact():
    """(K_lam, K_mu) exact for h = 1: K_e = h (lam K_lam + mu K_mu)."""
    if "ovfem" not in _CACHE:
        _CACHE["ovfem"] = (ovfem_stiffness_exact(1, 0), ovfem_stiffness_exact(0, 1))
    return _CACHE["ovfem"]


def ovfem_reference():
    """(K_lam, K_mu) as float64 arrays (exact values rounded once)."""
    Kl, Km = ovfem_reference_exact()
    return (np.array([[float(x) for x in r] for r in Kl]),
            np.array([[float(x) for x in r] for r in Km]))


def ovfem_mass_exact(rho=Fraction(1), h=Fraction(1)):
    """Element mass matrix of Eq. (6), rho (phi^a phi^a')_e, per node (8 x 8), exact.

    The octant indicators of distinct nodes do not overlap, so the matrix is
    diagonal; each diagonal entry is rho * (h/2)^3 * (volume of one octant in r).
    """
    h = Fraction(h)
    M = [[Fraction(0)] * 8 for _ in range(8)]
    for a in range(8):
        ra = node_rbar(a)
        for b in range(8):
            rb = node_rbar(b)
            v = Fraction(rho) * (h / 2) ** 3
            for k in range(3):
                # int_{-1}^{1} H(ra_k r) H(rb_k r) dr: 1 if same side, 0 otherwise
                v *= Fraction(1) if ra[k] == rb[k] else Fraction(0)
            M[a][b] = v
    return M


# ----------------------------------------------------------------------------------
# conventional trilinear voxel element (VFEM), for the dispersion comparison only

def trilinear_stiffness(lam, mu, h=1.0):
    """Trilinear hexahedron stiffness with 2x2x2 Gauss integration (float64, 24 x 24)."""
    g = 1.0 / np.sqrt(3.0)
    C = np.array(voigt_stiffness(float(lam), float(mu)), dtype=np.float64)
    K = np.zeros((24, 24))
    for gp in itertools.product((-g, g), repeat=3):
        dN = np.zeros((3, 8))  # d N_alpha / d x_j at the Gauss point
        for alpha in range(8):
            rb = node_rbar(alpha)
            f = [(1 + rb[k] * gp[k]) for k in range(3)]
            for j in range(3):
                d = rb[j]
                for k in range(3):
                    if k != j:
                        d *= f[k]
                dN[j, alpha] = d / 8.0 * (2.0 / h)
        B = np.zeros((6, 24))
        for v, (p, q) in enumerate(VOIGT):
            for alpha in range(8):
                if p == q:
                    B[v, 3 * alpha + p] += dN[p, alpha]
                else:
                    B[v, 3 * alpha + p] += dN[q, alpha]
                    B[v, 3 * alpha + q] += dN[p, alpha]
        K += B.T @ C @ B * (h / 2.0) ** 3  # unit Gauss weights
    return K


def trilinear_reference():
    """(K_lam, K_mu) of the trilinear element for h = 1 (float64): K_e = h (lam K_lam + mu K_mu)."""
    if "trilinear" not in _CACHE:
        _CACHE["trilinear"] = (trilinear_stiffness(1.0, 0.0, 1.0), trilinear_stiffness(0.0, 1.0, 1.0))
    return _CACHE["trilinear"]
