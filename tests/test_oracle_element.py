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
