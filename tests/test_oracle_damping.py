"""Oracle pins of the Rayleigh-damped stepper (C = alpha M + beta K).

The time discretization is a reading (the paper only says Rayleigh damping is used),
so the pins come from mathematics the reading must reproduce: the damping ratio of the
Rayleigh coefficients, the undamped special case, and the continuum limit of one
normal mode, whose amplitude decays as exp(-zeta w t) with zeta = alpha/(2w) + beta w/2
(first order in dt with the backward stiffness term, second order without it).
"""
import numpy as np
import pytest

from oracle import assembly as oasm
from paper_2404_13683_amd import workloads as wl


def test_rayleigh_coefficients_hit_the_damping_ratio_at_both_frequencies():
    zeta, f1, f2 = 0.05, 100e3, 125e3
    a, b = oasm.rayleigh_coefficients(zeta, f1, f2)
    for f in (f1, f2):
        w = 2 * np.pi * f
        assert a / (2 * w) + b * w / 2 == pytest.approx(zeta, rel=1e-14)
    w = 2 * np.pi * 0.5 * (f1 + f2)
    assert a / (2 * w) + b * w / 2 < zeta  # the ratio dips between the two frequencies


def _box(nx=4, ny=3, nz=3, seed=1):
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = rng.uniform(1800, 2400, shape)
    vs = rng.uniform(600, 900, shape)
    lam, mu = wl.lame_from_velocities(2 * vs, vs, rho)
    return lam, mu, rho, 1.0, wl.box_fixed(nx, ny, nz)


def _lowest_mode(lam, mu, rho, h, fixed):
    """Lowest generalized eigenpair (w^2, phi) of K phi = w^2 M phi on the free DOFs."""
    m0 = oasm.Model(lam, mu, rho, h, fixed, 1.0)
    K = oasm.dense_stiffness(lam, mu, h)
    free = np.repeat(m0.free.reshape(-1), 3)
    mass = np.repeat(m0.mass.reshape(-1), 3)[free]
    Kf = K[np.ix_(free, free)]
    s = 1.0 / np.sqrt(mass)
    w2, V = np.linalg.eigh(s[:, None] * Kf * s[None, :])
    phi = np.zeros(free.size)
    phi[free] = s * V[:, 0]
    return w2[0], phi.reshape(m0.node_shape)


def _decay_exponent(lam, mu, rho, h, fixed, alpha, beta, dt, T):
    """Decay rate of the lowest mode under the oracle's damped stepper, from rest at phi.

    u^n stays a multiple a_n of the mode, and a_n obeys some two-term linear recurrence
    whose roots z, conj(z) carry the decay; the Casoratian a_{n+1} a_{n-1} - a_n^2 of
    any such recurrence is proportional to |z|^(2n), so the rate -log|z| / dt is read
    off without assuming the scheme's coefficients."""
    m = oasm.Model(lam, mu, rho, h, fixed, dt, alpha=alpha, beta=beta)
    w2, phi = _lowest_mode(lam, mu, rho, h, fixed)
    Mphi = m.mass[..., None] * phi
    norm = float(np.sum(Mphi * phi))
    u, up = phi.copy(), phi.copy()
    n = int(round(T / dt))
    zero = np.zeros(m.node_shape)
    a = [1.0]
    for _ in range(n):
        un = m.step(u, up, zero)
        up, u = u, un
        a.append(float(np.sum(Mphi * u)) / norm)
    a = np.array(a)
    cas = a[2:] * a[:-2] - a[1:-1] ** 2
    k0, k1 = 10, len(cas) - 1
    return -np.log(cas[k1] / cas[k0]) / (2 * (k1 - k0) * dt), np.sqrt(w2)


def test_undamped_special_case_is_the_plain_step():
    lam, mu, rho, h, fixed = _box()
    rng = np.random.default_rng(3)
    m0 = oasm.Model(lam, mu, rho, h, fixed, 1e-4)
    m1 = oasm.Model(lam, mu, rho, h, fixed, 1e-4, alpha=0.0, beta=0.0)
    u, up, F = (rng.standard_normal(m0.node_shape) for _ in range(3))
    assert np.array_equal(m0.step(u, up, F), m1.step(u, up, F))


@pytest.mark.parametrize("kind", ["mass", "stiffness", "both"])
def test_modal_decay_converges_to_the_continuum_rate(kind):
    lam, mu, rho, h, fixed = _box()
    w2, _ = _lowest_mode(lam, mu, rho, h, fixed)
    w = np.sqrt(w2)
    zeta = 0.05
    alpha, beta = {"mass": (2 * zeta * w, 0.0), "stiffness": (0.0, 2 * zeta / w),
                   "both": (zeta * w, zeta / w)}[kind]
    exact = (alpha / (2 * w) + beta * w / 2) * w  # zeta w of the continuous oscillator
    T = 5 * 2 * np.pi / w
    errs = []
    for dt in (0.04 / w, 0.02 / w):
        rate, _ = _decay_exponent(lam, mu, rho, h, fixed, alpha, beta, dt, T)
        errs.append(abs(rate - exact) / exact)
    print(kind, "relative rate errors", errs)
    if kind == "mass":
        # centred mass term: second order, tiny at these steps
        assert errs[1] < 1e-5 and errs[0] / errs[1] > 3.0
    else:
        # backward stiffness term: first order, error close to the stiffness share of zeta w dt
        assert errs[1] < 2e-3
        assert 1.7 < errs[0] / errs[1] < 2.3


def _highest_mode(lam, mu, rho, h, fixed):
    """Highest generalized eigenpair (w^2, phi) of K phi = w^2 M phi on the free DOFs."""
    m0 = oasm.Model(lam, mu, rho, h, fixed, 1.0)
    K = oasm.dense_stiffness(lam, mu, h)
    free = np.repeat(m0.free.reshape(-1), 3)
    mass = np.repeat(m0.mass.reshape(-1), 3)[free]
    s = 1.0 / np.sqrt(mass)
    w2, V = np.linalg.eigh(s[:, None] * K[np.ix_(free, free)] * s[None, :])
    phi = np.zeros(free.size)
    phi[free] = s * V[:, -1]
    return w2[-1], phi.reshape(m0.node_shape)


@pytest.mark.parametrize("side", [0.98, 1.02])
def test_damped_stability_bound(side):
    """The damped step is stable exactly while w_max^2 dt (dt + 2 beta) <= 4 (the
    Jury conditions of the modal recurrence; independent of alpha >= 0): started on the
    highest mode, 2 % below that dt the mode stays bounded, 2 % above it grows."""
    lam, mu, rho, h, fixed = _box()
    w2, phi = _highest_mode(lam, mu, rho, h, fixed)
    w = np.sqrt(w2)
    beta = 0.3 / w
    alpha = 0.02 * w
    dt = side * (-beta + np.sqrt(beta * beta + 4.0 / w2))
    m = oasm.Model(lam, mu, rho, h, fixed, dt, alpha=alpha, beta=beta)
    Mphi = m.mass[..., None] * phi
    norm = float(np.sum(Mphi * phi))
    u, up = phi.copy(), phi.copy()
    zero = np.zeros(m.node_shape)
    amp = []
    for _ in range(3000):
        un = m.step(u, up, zero)
        up, u = u, un
        amp.append(abs(float(np.sum(Mphi * u)) / norm))
    print("side %.2f: |a| after 100, 1000, 3000 steps: %.3e %.3e %.3e" % (side, amp[99], amp[999], amp[-1]))
    if side < 1.0:
        assert max(amp) < 2.0
    else:
        assert amp[-1] > 1e3 and amp[-1] > 100 * amp[999]
