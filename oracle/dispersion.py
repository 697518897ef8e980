"""Plane-wave (Bloch) analysis of the assembled voxel operators (oracle; tests only).

On an infinite homogeneous grid the assembled operator is translation invariant, so
a plane wave u_n = U exp(i k . x_n) is an eigenvector family: K u = S(k) u with the
3 x 3 Hermitian symbol

    S(k) = sum over the 8 elements around node 0 of
           sum_{alpha'} K_e[node-0 block, alpha' block] exp(i k . (x_alpha' - x_0)).

With the diagonal nodal mass m = rho h^3 (eight octants of rho h^3 / 8), the
semi-discrete dispersion relation is omega^2 m U = S(k) U, whose three eigenvalues
give one quasi-P and two quasi-S branches.  Phase velocity c_h = omega / |k|.
This quantifies the numerical dispersion that Sec. 2 attributes to the lumped
trilinear element and claims OVFEM suppresses.
"""
import numpy as np


def bloch_symbol(Ke, h, kvec):
    """S(k) for element matrix Ke (24 x 24, DOF 3 alpha + c) on a grid of spacing h."""
    S = np.zeros((3, 3), dtype=np.complex128)
    k = np.asarray(kvec, dtype=np.float64)
    for alpha0 in range(8):  # node 0 is corner alpha0 of this element
        o = np.array([alpha0 & 1, (alpha0 >> 1) & 1, (alpha0 >> 2) & 1])
        for alpha in range(8):
            p = np.array([alpha & 1, (alpha >> 1) & 1, (alpha >> 2) & 1])
            phase = np.exp(1j * h * np.dot(k, p - o))
            S += Ke[3 * alpha0:3 * alpha0 + 3, 3 * alpha:3 * alpha + 3] * phase
    return S


def phase_velocities(Ke, rho, h, direction, kh):
    """Sorted phase velocities (slowest first) for wave number |k| = kh / h along direction."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    k = d * (kh / h)
    S = bloch_symbol(Ke, h, k)
    w2 = np.linalg.eigvalsh(0.5 * (S + S.conj().T)) / (rho * h ** 3)
    w = np.sqrt(np.clip(w2, 0.0, None))
    return np.sort(w / (kh / h))


def max_frequency(Ke, rho, h, n=24):
    """Largest omega over a grid of the Brillouin zone (for the stability limit dt < 2/omega_max)."""
    best = 0.0
    ks = np.linspace(-np.pi, np.pi, n + 1)
    for a in ks:
        for b in ks:
            for c in ks:
                S = bloch_symbol(Ke, h, np.array([a, b, c]) / h)
                w2 = np.linalg.eigvalsh(0.5 * (S + S.conj().T)).max() / (rho * h ** 3)
                best = max(best, np.sqrt(max(w2, 0.0)))
    return best
