"""GPU parity at the full workload sizes, on outputs the oracle computes one by one.

At these sizes the oracle cannot run whole simulations inside a test, so each case is
checked three ways:
  * K u on the full mesh, against the oracle's K u at sampled nodes (seeded random nodes
    plus nodes on tile, chunk and domain boundaries), relative L2 over the sample <= 1e-12;
  * one time step taken from the GPU's own state after many steps, against the oracle's
    update at the sampled nodes (the same tolerance);
  * the INT8 path against the FP64 path over all steps of the run, traces within 1e-9
    (the FP64 path is pinned to the oracle over whole runs at smaller sizes).
The launch configuration is the autotuned one that bench.py times.
"""
import numpy as np
import pytest

from oracle import assembly as oasm
from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu

MATVEC_TOL = 1e-12
TRACE_TOL = 1e-9


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def sample_nodes(w, n_random=300, seed=0):
    """(k, j, i) triples: seeded random nodes, nodes next to every 15-node tile edge in x
    and y and to several z-chunk depths, the grid's corners and face centres, and the
    source and receiver nodes."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = w.nx, w.ny, w.nz
    pts = set()
    for _ in range(n_random):
        pts.add((int(rng.integers(0, nz + 1)), int(rng.integers(0, ny + 1)), int(rng.integers(0, nx + 1))))
    for edge in range(0, max(nx, ny) + 1, 15):
        for d in (-1, 0, 1):
            for planes in (8, 12, 16, 24, 32):
                k = min(nz, max(0, (int(rng.integers(1, nz // planes + 2)) * planes + d)))
                if 0 <= edge + d <= nx:
                    pts.add((k, int(rng.integers(0, ny + 1)), edge + d))
                if 0 <= edge + d <= ny:
                    pts.add((k, edge + d, int(rng.integers(0, nx + 1))))
    for k in (0, nz // 2, nz):
        for j in (0, ny // 2, ny):
            for i in (0, nx // 2, nx):
                pts.add((k, j, i))
    for nd in list(w.src_node) + list(w.rec_node):
        nd = int(nd)
        pts.add((nd // ((nx + 1) * (ny + 1)), (nd // (nx + 1)) % (ny + 1), nd % (nx + 1)))
    return sorted(pts)


def _flat(w, pts):
    return np.array([i + (w.nx + 1) * (j + (w.ny + 1) * k) for k, j, i in pts], np.int64)


def _solid(w):
    return None if w.solid is None else w.solid.astype(bool)


def check_matvec_sampled(w, solver, prec, seed=5):
    import torch
    shape = (w.nz + 1, w.ny + 1, w.nx + 1, 3)
    # a smooth long-wavelength field plus a small random part: K u then has the
    # cancellation of a real wavefield
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(w.nz + 1), np.arange(w.ny + 1), np.arange(w.nx + 1), indexing="ij")
    u = np.empty(shape)
    for c in range(3):
        kx, ky, kz = rng.uniform(0.01, 0.1, 3)
        u[..., c] = np.sin(kx * x + ky * y + kz * z + c)
    del x, y, z
    u += 1e-3 * rng.standard_normal(shape)
    ut = torch.from_numpy(u.reshape(-1)).cuda()
    ku = solver.matvec(ut)
    pts = sample_nodes(w, seed=seed)
    idx = torch.from_numpy(_flat(w, pts)).cuda()
    got = ku.view(-1, 3).index_select(0, idx).cpu().numpy()
    ref = oasm.matvec_at_nodes(u, w.lam, w.mu, w.h, pts, solid=_solid(w))
    err = _rel(got, ref)
    print("%s %s sampled matvec (%d nodes) rel L2 %.3e" % (w.name, prec, len(pts), err))
    assert err <= MATVEC_TOL


def check_one_step_sampled(w, solver, prec, shot=0):
    """Take one more step on the GPU and compare u^{n+1} at sampled nodes with the
    oracle's update from the GPU's own (u^n, u^{n-1})."""
    n = solver.get_step()
    nn = w.n_nodes
    un = solver.get_wavefield(0).view(-1, nn, 3)[shot].cpu().numpy().reshape(w.nz + 1, w.ny + 1, w.nx + 1, 3)
    um = solver.get_wavefield(1).view(-1, nn, 3)[shot].cpu().numpy().reshape(un.shape)
    solver.step(1)
    pts = sample_nodes(w, n_random=200, seed=n)
    flat = _flat(w, pts)
    got = solver.get_wavefield(0).view(-1, nn, 3)[shot].cpu().numpy()[flat]
    ku = oasm.matvec_at_nodes(un, w.lam, w.mu, w.h, pts, solid=_solid(w))
    mass = oasm.nodal_mass(w.rho, w.h, _solid(w))
    free = oasm.free_mask(w.fixed, mass)
    sel = np.asarray(w.src_shot) == shot
    F = np.zeros((len(pts), 3))
    for nd, c, row in zip(w.src_node[sel], w.src_comp[sel], w.wavelet[sel]):
        hit = np.nonzero(flat == nd)[0]
        if hit.size and n < row.shape[0]:
            F[hit, c] += row[n]
    ref = np.zeros((len(pts), 3))
    for r, (k, j, i) in enumerate(pts):
        if free[k, j, i]:
            a = w.dt ** 2 / mass[k, j, i]
            ref[r] = 2.0 * un[k, j, i] - um[k, j, i] + a * (F[r] - ku[r])
    err = _rel(got, ref)
    print("%s %s one step at %d sampled nodes after %d steps: rel L2 %.3e" % (w.name, prec, len(pts), n, err))
    assert err <= MATVEC_TOL


def run_pair(w, steps, check_state_after=None):
    """Both paths over `steps` steps (autotuned launch configuration); returns traces."""
    from paper_2404_13683_amd.ovfem import Solver
    out = {}
    for prec in ("fp64", "int8", "fp64-sf"):
        s = Solver.from_workload(w, precision=prec, receivers_nt=steps + 1)
        s.autotune(steps=6)
        check_matvec_sampled(w, s, prec)
        s.reset()
        s.step(steps)
        out[prec] = s.get_traces().cpu().numpy()[..., :steps]
        if check_state_after:
            check_one_step_sampled(w, s, prec)
        s.close()
    for p in ("int8", "fp64-sf"):
        err = _rel(out[p], out["fp64"])
        print("%s %s vs FP64 traces over %d steps: rel L2 %.3e" % (w.name, p, steps, err))
        assert err <= TRACE_TOL
    return out


@pytest.mark.timeout(600)
def test_c2_layered_256x256x128_2000_steps():
    w = wl.layered_c2()
    run_pair(w, w.nt, check_state_after=True)


@pytest.mark.timeout(900)
def test_c5_topography_512x512x256_4000_steps():
    w = wl.topography_c5()
    run_pair(w, w.nt, check_state_after=True)


@pytest.mark.timeout(600)
def test_c5_slab_512x512x32_4000_steps_both_tile_heights():
    """The 512 x 512 x 32 slab of the topography recipe (one GPU's share of the large model
    split eight ways along z), where the tuner prefers the 16 x 32-element tiles: both tile
    heights against the oracle at sampled nodes, and against the FP64 path over all steps."""
    from paper_2404_13683_amd.ovfem import Solver
    w = wl.topography_c5(nz=32)
    out = run_pair(w, w.nt, check_state_after=True)
    for rows, planes in ((32, 12), (16, 32)):
        s = Solver.from_workload(w, precision="int8", receivers_nt=w.nt + 1)
        s.set_tuning(chunk_planes=planes, tile_rows=rows)
        assert s.get_tuning()["tile_rows"] == rows
        check_matvec_sampled(w, s, "int8 rows=%d" % rows)
        s.reset()
        s.step(w.nt)
        tr = s.get_traces().cpu().numpy()[..., :w.nt]
        err = _rel(tr, out["fp64"])
        print("%s int8 tile rows %d, %d planes vs FP64 traces: rel L2 %.3e" % (w.name, rows, planes, err))
        assert err <= TRACE_TOL
        check_one_step_sampled(w, s, "int8 rows=%d" % rows)
        s.close()


@pytest.mark.timeout(600)
def test_c3_64_shots_128x128x64_1000_steps():
    """All 64 shots in one solver; two of them against one-shot solvers (bitwise) and
    against the oracle's update at sampled nodes."""
    from paper_2404_13683_amd.ovfem import Solver
    w = wl.shots_c3()
    s = Solver.from_workload(w, precision="int8")
    s.autotune(steps=4)
    tuning = s.get_tuning()
    s.reset()
    s.step(w.nt)
    tr = s.get_traces().cpu().numpy()
    u = s.get_wavefield(0).view(w.n_shots, -1).cpu().numpy()
    for k in (0, 41):
        one = Solver.from_workload(wl.single_shot(w, k), precision="int8")
        one.set_tuning(chunk_planes=tuning["chunk_planes"], tile_rows=tuning["tile_rows"])
        one.step(w.nt)
        assert np.array_equal(one.get_traces().cpu().numpy()[0], tr[k]), k
        assert np.array_equal(one.get_wavefield(0).cpu().numpy(), u[k]), k
        one.close()
    f = Solver.from_workload(wl.single_shot(w, 41), precision="fp64")
    f.step(w.nt)
    err = _rel(tr[41], f.get_traces().cpu().numpy()[0])
    print("c3 shot 41 INT8 (batched) vs FP64: %.3e" % err)
    assert err <= TRACE_TOL
    f.close()
    check_one_step_sampled(w, s, "int8", shot=41)
    s.close()


@pytest.mark.timeout(600)
def test_c3_16_uneven_domains_1000_steps():
    from paper_2404_13683_amd.ovfem import Batch, Solver
    doms = wl.uneven_domains_c3()
    members = [Solver.from_workload(d, precision="int8") for d in doms]
    b = Batch(members)
    b.step(doms[0].nt)
    b.close()
    for k in (0, 7, 15):
        alone = Solver.from_workload(doms[k], precision="int8")
        alone.step(doms[k].nt)
        assert np.array_equal(alone.get_traces().cpu().numpy(), members[k].get_traces().cpu().numpy()), k
        alone.close()
        f = Solver.from_workload(doms[k], precision="fp64")
        f.step(doms[k].nt)
        err = _rel(members[k].get_traces().cpu().numpy(), f.get_traces().cpu().numpy())
        print("uneven domain %d (%dx%dx%d) INT8 batch vs FP64: %.3e" % (k, doms[k].nx, doms[k].ny, doms[k].nz, err))
        assert err <= TRACE_TOL
        f.close()
    check_one_step_sampled(doms[15], members[15], "int8")


@pytest.mark.timeout(600)
def test_c4_adjoint_96cubed_1000_steps_central_differences():
    """Adjoint workload at full size: 96^3, 1000 steps, checkpoints every 50; gradient
    against central differences (eps = 1e-3 of the local value) on 20 seeded voxels with
    |g| >= 1e-2 max |g| (10 for lam, 10 for mu), and the INT8 gradient against FP64."""
    from paper_2404_13683_amd.ovfem import Solver
    true, start = wl.adjoint_c4()
    s = Solver.from_workload(true, precision="fp64")
    s.step(true.nt)
    d_obs = s.get_traces().clone()
    s.close()
    grads = {}
    for prec in ("fp64", "int8"):
        s = Solver.from_workload(start, precision=prec)
        s.set_checkpointing(50, start.nt)
        s.step(start.nt)
        res = (s.get_traces() - d_obs).contiguous()
        grads[prec] = [g.cpu().numpy() for g in s.adjoint(res)]
        s.close()
    for a, b in zip(grads["int8"], grads["fp64"]):
        err = _rel(a, b)
        print("c4 INT8 vs FP64 gradient rel L2 %.3e" % err)
        assert err <= TRACE_TOL
    s = Solver.from_workload(start, precision="fp64")

    def J(lam, mu):
        s.set_model(lam, mu, start.rho)
        s.set_dt(start.dt)
        s.step(start.nt)
        r = (s.get_traces() - d_obs).cpu().numpy()
        return 0.5 * float(np.sum(r * r))

    rng = np.random.default_rng(20)
    checked = 0
    for which, g in zip(("lam", "mu"), grads["fp64"]):
        cand = np.argwhere(np.abs(g) >= 1e-2 * np.abs(g).max())
        for idx in cand[rng.choice(len(cand), size=10, replace=False)]:
            k, j, i = map(int, idx)
            lam, mu = start.lam.copy(), start.mu.copy()
            arr = lam if which == "lam" else mu
            base = arr[k, j, i]
            eps = 1e-3 * base
            arr[k, j, i] = base + eps
            jp = J(lam, mu)
            arr[k, j, i] = base - eps
            jm = J(lam, mu)
            fd = (jp - jm) / (2 * eps)
            print("c4 FD %s %s: adjoint %.8e fd %.8e rel %.2e" % (which, (k, j, i), g[k, j, i], fd,
                                                                 abs(g[k, j, i] - fd) / abs(fd)))
            assert abs(g[k, j, i] - fd) <= 1e-4 * abs(fd)
            checked += 1
    assert checked == 20
    s.close()
