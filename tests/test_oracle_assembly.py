"""Pins of the oracle's assembled operator: brute force, patch test, Navier consistency."""
import numpy as np
import pytest

from oracle import assembly as asm


def _grid_coords(nx, ny, nz, h):
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    return i * h, j * h, k * h


def test_slice_matvec_equals_plain_loop_assembly():
    rng = np.random.default_rng(0)
    nx, ny, nz, h = 3, 2, 2, 0.7
    lam = rng.uniform(1, 3, (nz, ny, nx))
    mu = rng.uniform(1, 3, (nz, ny, nx))
    u = rng.standard_normal((nz + 1, ny + 1, nx + 1, 3))
    K = asm.dense_stiffness(lam, mu, h)
    f_dense = (K @ u.reshape(-1)).reshape(u.shape)
    f = asm.matvec(u, lam, mu, h)
    assert np.abs(f - f_dense).max() <= 1e-13 * np.abs(f_dense).max()
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())


def test_assembled_operator_symmetric_heterogeneous():
    rng = np.random.default_rng(1)
    nx, ny, nz, h = 5, 4, 3, 2.0
    lam = rng.uniform(0.5, 4, (nz, ny, nx))
    mu = rng.uniform(0.5, 4, (nz, ny, nx))
    u = rng.standard_normal((nz + 1, ny + 1, nx + 1, 3))
    v = rng.standard_normal((nz + 1, ny + 1, nx + 1, 3))
    a = np.sum(v * asm.matvec(u, lam, mu, h))
    b = np.sum(u * asm.matvec(v, lam, mu, h))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_patch_test_linear_fields_give_zero_interior_force():
    nx, ny, nz, h = 6, 5, 4, 1.3
    lam = np.full((nz, ny, nx), 2.5)
    mu = np.full((nz, ny, nx), 1.1)
    x, y, z = _grid_coords(nx, ny, nz, h)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    u = np.stack([A[c, 0] * x + A[c, 1] * y + A[c, 2] * z + b[c] for c in range(3)], -1)
    f = asm.matvec(u, lam, mu, h)
    scale = h * (2.5 + 2 * 1.1) * np.abs(u).max() * 8
    assert np.abs(f[1:-1, 1:-1, 1:-1]).max() <= 1e-13 * scale


@pytest.mark.parametrize("field,comp,expect", [
    ("xx", 0, "lam+2mu"),  # u_x = x^2/2  -> -(Ku)_x / h^3 = lam + 2 mu
    ("yy", 0, "mu"),       # u_x = y^2/2  -> mu
    ("xy", 1, "lam+mu"),   # u_x = x y    -> (Ku)_y picks lam + mu
])
def test_navier_consistency_on_quadratic_fields(field, comp, expect):
    """Interior rows of K reproduce -div(c : grad u) h^3 exactly for quadratic u.

    Continuum: for u_x = x^2/2 the stress sigma_11 = (lam + 2 mu) x, so the body force
    in equilibrium is -(lam + 2 mu) e_x; the consistent nodal force of the dual cell
    (volume h^3) is that times h^3.
    """
    nx, ny, nz, h = 6, 6, 6, 0.9
    lam0, mu0 = 2.7, 1.3
    lam = np.full((nz, ny, nx), lam0)
    mu = np.full((nz, ny, nx), mu0)
    x, y, z = _grid_coords(nx, ny, nz, h)
    u = np.zeros((nz + 1, ny + 1, nx + 1, 3))
    if field == "xx":
        u[..., 0] = 0.5 * x * x
    elif field == "yy":
        u[..., 0] = 0.5 * y * y
    else:
        u[..., 0] = x * y
    f = asm.matvec(u, lam, mu, h)
    want = {"lam+2mu": lam0 + 2 * mu0, "mu": mu0, "lam+mu": lam0 + mu0}[expect]
    inner = -f[1:-1, 1:-1, 1:-1, comp] / h ** 3
    assert np.abs(inner - want).max() <= 1e-11 * want
    other = [c for c in range(3) if c != comp]
    assert np.abs(f[1:-1, 1:-1, 1:-1][..., other]).max() <= 1e-11 * want * h ** 3


def test_nodal_mass_counts_eighths():
    nx, ny, nz, h = 4, 3, 2, 2.0
    rng = np.random.default_rng(3)
    rho = rng.uniform(1, 2, (nz, ny, nx))
    m = asm.nodal_mass(rho, h)
    assert abs(m.sum() - rho.sum() * h ** 3) <= 1e-12 * m.sum()
    # interior node of a homogeneous block gets the whole dual-cell mass rho h^3
    m2 = asm.nodal_mass(np.full((4, 4, 4), 3.0), 0.5)
    assert m2[2, 2, 2] == 3.0 * 0.125
    assert m2[0, 0, 0] == 3.0 * 0.125 / 8


def test_removed_voxels_carry_no_stiffness_or_mass():
    rng = np.random.default_rng(5)
    nx, ny, nz, h = 3, 3, 3, 1.0
    lam = rng.uniform(1, 2, (nz, ny, nx))
    mu = rng.uniform(1, 2, (nz, ny, nx))
    rho = np.ones((nz, ny, nx))
    solid = np.ones((nz, ny, nx), bool)
    solid[2, :, :2] = False
    m = asm.Model(lam, mu, rho, h, np.zeros((nz + 1, ny + 1, nx + 1), np.uint8), 0.1, solid)
    lam2 = np.where(solid, lam, 0.0)
    mu2 = np.where(solid, mu, 0.0)
    u = rng.standard_normal((nz + 1, ny + 1, nx + 1, 3))
    assert np.array_equal(m.K(u), asm.matvec(u, lam2, mu2, h))
    # a node touched only by removed voxels has no mass and is not free
    assert m.mass[3, 3, 0] == 0 and not m.free[3, 3, 0]


def test_err_measure_definition():
    ref = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 1.0]])
    assert asm.err_measure(ref, ref) == 0.0
    assert asm.err_measure(2 * ref, ref) == pytest.approx(1.0)
    obs = ref.copy()
    obs[0, 1] += 1.0
    # channel 0: 1 / 5, channel 1: 0  -> mean 0.1
    assert asm.err_measure(obs, ref) == pytest.approx(0.1)


@pytest.mark.parametrize("shape", [(5, 4, 3), (1, 1, 1), (2, 1, 3), (4, 4, 4)])
def test_sampled_matvec_equals_the_assembled_matvec_at_every_node(shape):
    """matvec_at_nodes, the per-node loop that checks full-size results on sampled outputs,
    gives (K u) of the assembled operator (Sec. 2, Eqs. (2) and (5)) at every node of
    small grids: every corner, edge, face and interior node, with voxels removed.  It is
    checked against Model.K (slice assembly, itself pinned to the plain-loop dense matrix)
    and, on the smallest grids, against the dense matrix directly."""
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    h = 0.9
    lam = rng.uniform(1, 3, (nz, ny, nx))
    mu = rng.uniform(1, 3, (nz, ny, nx))
    rho = rng.uniform(1, 2, (nz, ny, nx))
    solid = rng.uniform(size=(nz, ny, nx)) > 0.3
    if solid.size > 1:
        solid.flat[0] = False  # a hole at a grid corner, whatever the draw
    u = rng.standard_normal((nz + 1, ny + 1, nx + 1, 3))
    model = asm.Model(lam, mu, rho, h, np.zeros((nz + 1, ny + 1, nx + 1), np.uint8), 1.0, solid=solid)
    ref = model.K(u)
    nodes = [(k, j, i) for k in range(nz + 1) for j in range(ny + 1) for i in range(nx + 1)]
    got = asm.matvec_at_nodes(u, lam, mu, h, nodes, solid=solid)
    want = np.array([ref[k, j, i] for k, j, i in nodes])
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 1e-14 * scale
    # the unmasked arrays with the mask given, and the masked arrays without it, agree
    got2 = asm.matvec_at_nodes(u, model.lam, model.mu, h, nodes)
    assert np.abs(got2 - want).max() <= 1e-14 * scale
    if nx * ny * nz <= 12:
        K = asm.dense_stiffness(model.lam, model.mu, h)
        dense = (K @ u.reshape(-1)).reshape(-1, 3)
        flat = [i + (nx + 1) * (j + (ny + 1) * k) for k, j, i in nodes]
        assert np.abs(got - dense[flat]).max() <= 1e-13 * scale
    # a removed voxel is really left out: unmasked lam/mu give a different answer
    if not solid.all():
        full = asm.matvec_at_nodes(u, lam, mu, h, nodes)
        assert np.abs(full - want).max() > 1e-6 * scale
