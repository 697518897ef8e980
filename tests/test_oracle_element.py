"""Pins of the oracle's element matrices against the paper and elementary mechanics.

Each test targets a plausible mistake: a wrong basis integral, a wrong Voigt
row, a missing 1/3 in the psi Gram matrix, a transposed block.
"""
import json
import os
from fractions import Fraction

import numpy as np

from oracle import element as el

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_claims.json")))


def _rigid_modes(h=Fraction(1)):
    """Three translations and three infinitesimal rotations sampled at the 8 corners (exact)."""
    modes = []
    for c in range(3):
        v = [Fraction(0)] * 24
        for a in range(8):
            v[3 * a + c] = Fraction(1)
        modes.append(v)
    for axis in range(3):
        w = [0, 0, 0]
        w[axis] = 1
        v = [Fraction(0)] * 24
        for a in range(8):
            x = [Fraction(s) * h / 2 for s in el.node_rbar(a)]
            r = (w[1] * x[2] - w[2] * x[1], w[2] * x[0] - w[0] * x[2], w[0] * x[1] - w[1] * x[0])
            for c in range(3):
                v[3 * a + c] = r[c]
        modes.append(v)
    return modes


def test_element_mass_is_diagonal_with_eighth_of_voxel_mass():
    # Sec. 2 after Eq. (8): with Eq. (7) the element mass of Eq. (6) is diagonal
    rho, h = Fraction(7, 3), Fraction(5, 2)
    M = el.ovfem_mass_exact(rho, h)
    for a in range(8):
        for b in range(8):
            assert M[a][b] == (rho * h ** 3 / 8 if a == b else 0)
    assert sum(M[a][a] for a in range(8)) == rho * h ** 3   # total voxel mass


def test_psi_basis_orthogonal_and_normalised():
    # Eq. (8) monomials are orthogonal on the voxel; |psi|^2 = h^3 3^-degree
    h = Fraction(3)
    P = el.psi_gram(h)
    for b, ab in enumerate(el.PSI_EXPONENTS):
        for bp in range(7):
            expect = h ** 3 / Fraction(3) ** sum(ab) if b == bp else 0
            assert P[b][bp] == expect
    assert len(el.PSI_EXPONENTS) == GOLDEN["stress_basis_size"]["value"]


def test_stiffness_symmetric_exact():
    Kl, Km = el.ovfem_reference_exact()
    for K in (Kl, Km):
        for i in range(24):
            for j in range(24):
                assert K[i][j] == K[j][i]


def test_rigid_body_modes_in_null_space_exact():
    Kl, Km = el.ovfem_reference_exact()
    for v in _rigid_modes():
        for K in (Kl, Km):
            for i in range(24):
                assert sum(K[i][j] * v[j] for j in range(24)) == 0


def test_rank_is_18_and_positive_semidefinite():
    Kl, Km = el.ovfem_reference()
    for lam, mu in ((1.0, 1.0), (2.0, 1.0), (0.0, 1.0)):
        K = lam * Kl + mu * Km
        ev = np.linalg.eigvalsh(K)
        assert np.all(ev > -1e-13 * ev.max())
        assert np.linalg.matrix_rank(K, tol=1e-10 * ev.max()) == 18


def test_stiffness_scales_linearly_with_h():
    # K_e is proportional to h (Eq. (5): (psi grad phi) ~ h^2, (psi psi) ~ h^3)
    h = Fraction(3, 2)
    K2 = el.ovfem_stiffness_exact(1, 1, h)
    Kl, Km = el.ovfem_reference_exact()
    for i in range(24):
        for j in range(24):
            assert K2[i][j] == h * (Kl[i][j] + Km[i][j])


def test_paper_kint8_integer_and_in_int8_range():
    """Eq. (9) rearranged: K^kappa = 256 dK/dkappa / ds and Kbar^G = 384 dK/dG / ds - 128 I.

    Eq. (9) holds for every kappa, G only with these two matrices; the paper states
    that they are constant integer matrices inside the INT8 range.  With
    lam = kappa - 2G/3 and mu = G: dK/dkappa = ds K_lam, dK/dG = ds (K_mu - 2/3 K_lam).
    """
    Kl, Km = el.ovfem_reference_exact()
    lo, hi = GOLDEN["kint8_entry_range"]["value"]
    rows = []
    for i in range(24):
        kk = [256 * Kl[i][j] for j in range(24)]
        kg = [384 * (Km[i][j] - Fraction(2, 3) * Kl[i][j]) - (128 if i == j else 0) for j in range(24)]
        rows.append(kk + kg)
    assert [len(rows), len(rows[0])] == GOLDEN["kint8_shape"]["value"]
    for r in rows:
        for x in r:
            assert x.denominator == 1, "K^INT8 entry is not an integer"
            assert lo <= x <= hi


def test_eq9_identity_reproduces_element_matvec():
    # Eq. (9): K_e u_e = (1/256) kappa ds (K^INT8 ubar_e + 256/3 G/kappa u_e),
    # ubar_e = (u_e, 2/3 G/kappa u_e)  -- exact rational check for one sample
    Kl, Km = el.ovfem_reference_exact()
    rng = np.random.default_rng(0)
    u = [Fraction(int(x), 97) for x in rng.integers(-1000, 1000, 24)]
    kappa, G, ds = Fraction(53, 7), Fraction(11, 5), Fraction(3, 2)
    lam, mu = kappa - Fraction(2, 3) * G, G
    Kint = [[256 * Kl[i][j] for j in range(24)]
            + [384 * (Km[i][j] - Fraction(2, 3) * Kl[i][j]) - (128 if i == j else 0) for j in range(24)]
            for i in range(24)]
    ubar = u + [Fraction(2, 3) * G / kappa * x for x in u]
    for i in range(24):
        lhs = ds * sum((lam * Kl[i][j] + mu * Km[i][j]) * u[j] for j in range(24))
        rhs = kappa * ds / 256 * (sum(Kint[i][j] * ubar[j] for j in range(48))
                                  + Fraction(256, 3) * G / kappa * u[i])
        assert lhs == rhs


def test_constant_strain_energy_matches_continuum():
    # a homogeneous strain field eps stored in one voxel has energy V/2 eps:c:eps
    Kl, Km = el.ovfem_reference()
    lam, mu, h = 3.0, 2.0, 1.0
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 3))
    E = 0.5 * (A + A.T)
    u = np.zeros(24)
    for a in range(8):
        x = np.array(el.node_rbar(a)) * h / 2
        u[3 * a:3 * a + 3] = E @ x
    Ke = h * (lam * Kl + mu * Km)
    energy = 0.5 * u @ Ke @ u
    cont = 0.5 * h ** 3 * (lam * np.trace(E) ** 2 + 2 * mu * np.sum(E * E))
    assert abs(energy - cont) <= 1e-13 * cont


def test_trilinear_element_sanity():
    K = el.trilinear_stiffness(2.0, 1.0, 1.0)
    assert np.allclose(K, K.T, atol=1e-13)
    ev = np.linalg.eigvalsh(K)
    assert np.linalg.matrix_rank(K, tol=1e-10 * ev.max()) == 18
    for v in _rigid_modes():
        assert np.abs(K @ np.array([float(x) for x in v])).max() < 1e-12


def _trilinear_closed_form():
    """Trilinear K_lam, K_mu (h = 1) from exact polynomial integrals, in rationals.

    With N_a = (1/8) prod_k (1 + s_ak r_k) on [-1, 1]^3 (x = (r + 1)/2):
      int dN_a/dr_i dN_b/dr_i = (1/64) s_ai s_bi * 2 * prod_{k != i} (2 + (2/3) s_ak s_bk),
      int dN_a/dr_i dN_b/dr_j = (1/64) s_ai s_bj * 2 * 2 * (2 + (2/3) s_al s_bl),  i != j, l the third axis,
    and d/dx = 2 d/dr, dx = dr / 8, so G_ij(a, b) = int dN_a/dx_i dN_b/dx_j dx = (1/2) * (r-integral).
    K_lam[3a+c][3b+d] = G_cd(a, b); K_mu[3a+c][3b+d] = delta_cd sum_k G_kk(a, b) + G_dc(a, b).
    """
    from fractions import Fraction as Fr
    s = [el.node_rbar(a) for a in range(8)]
    G = {}
    for a in range(8):
        for b in range(8):
            for i in range(3):
                for j in range(3):
                    if i == j:
                        v = Fr(2)
                        for k in range(3):
                            if k != i:
                                v *= 2 + Fr(2, 3) * s[a][k] * s[b][k]
                    else:
                        l = 3 - i - j
                        v = 4 * (2 + Fr(2, 3) * s[a][l] * s[b][l])
                    G[a, b, i, j] = Fr(1, 2) * Fr(1, 64) * s[a][i] * s[b][j] * v
    Kl = [[G[m // 3, n // 3, m % 3, n % 3] for n in range(24)] for m in range(24)]
    Km = [[(sum(G[m // 3, n // 3, k, k] for k in range(3)) if m % 3 == n % 3 else 0) + G[m // 3, n // 3, n % 3, m % 3]
           for n in range(24)] for m in range(24)]
    return Kl, Km


def test_trilinear_reference_equals_its_closed_form_and_is_72_integral():
    """The 2x2x2 Gauss integration is exact for the trilinear stiffness (polynomial of
    degree 2 per axis): the oracle's matrices equal the closed-form integrals, and
    72 K_lam, 72 K_mu are integer matrices (the INT8 scaling of this element)."""
    Kl, Km = el.trilinear_reference()
    Cl, Cm = _trilinear_closed_form()
    for K, C in ((Kl, Cl), (Km, Cm)):
        C = np.array([[float(x) for x in r] for r in C])
        assert np.abs(K - C).max() < 1e-15
        assert np.abs(72 * K - np.round(72 * K)).max() < 1e-12
    Cl, Cm = _trilinear_closed_form()
    assert all((72 * x).denominator == 1 for r in Cl + Cm for x in r)
    assert max(abs(72 * x) for r in Cl for x in r) == 8     # 72 K_lam in [-8, 8]
    assert max(abs(72 * x) for r in Cm for x in r) == 32    # diagonal of 72 K_mu
    # the known diagonal of the unit brick: K_lam[0][0] = 1/9, K_mu[0][0] = 4/9
    assert Cl[0][0] == Fraction(1, 9) and Cm[0][0] == Fraction(4, 9)


def test_trilinear_constant_strain_energy():
    """Patch test of the element: a linear field's strain energy equals the continuum's."""
    rng = np.random.default_rng(5)
    E = rng.standard_normal((3, 3))
    E = 0.5 * (E + E.T)
    h, lam, mu = 0.7, 2.3, 1.1
    Kl, Km = el.trilinear_reference()
    u = np.concatenate([h * (np.array(el.node_rbar(a)) + 1) / 2 @ E for a in range(8)])
    energy = 0.5 * u @ (h * (lam * Kl + mu * Km)) @ u
    cont = 0.5 * h ** 3 * (lam * np.trace(E) ** 2 + 2 * mu * np.sum(E * E))
    assert abs(energy - cont) <= 1e-13 * cont


def test_first_rows_of_the_integer_matrices():
    """Row 0 (corner 0, x component) of 256 K_lam and 128 K_mu, as integers: the values of a
    separate derivation of the element integrals with the same node numbering."""
    Kl, Km = el.ovfem_reference()
    row_l = [49, 28, 28, -49, 28, 28, 7, -28, 4, -7, -28, 4, 7, 4, -28, -7, 4, -28, 1, -4, -4, -1, -4, -4]
    row_m = [98, 14, 14, -42, -14, -14, -14, 14, 2, -10, -14, -2, -14, 2, 14, -10, -2, -14, -6, 2, 2, -2, -2, -2]
    assert np.array_equal(256 * Kl[0], np.array(row_l, dtype=float))
    assert np.array_equal(128 * Km[0], np.array(row_m, dtype=float))
    assert np.abs(256 * Kl[0]).sum() == 384
