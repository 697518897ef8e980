"""GPU: many shots per solver, batches of uneven grids, captured step graphs and the
launch tuner.

Every batched, captured or retuned form must reproduce the plain one-shot, one-launch-
per-step results bitwise in FP64 (the same kernels on the same tiles; the node sums are
order-independent).  Those plain runs are pinned to the oracle in the parity tests; a
shot of a batch and a topography run are compared with the oracle here as well.
"""
import numpy as np
import pytest

from oracle import assembly as oasm
from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "int8", "int8-bf16", "fp64-sf"]
TRACE_TOL = 1e-9


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _solver(w, prec, tile_rows=None, **tuning):
    from paper_2404_13683_amd.ovfem import Solver
    s = Solver.from_workload(w, precision=prec)
    if tile_rows is not None:
        s.set_tuning(**dict(s.get_tuning(), tile_rows=tile_rows, **tuning))
    elif tuning:
        s.set_tuning(**tuning)
    return s


def _state(s):
    return (s.get_wavefield(0).cpu().numpy(), s.get_wavefield(1).cpu().numpy(),
            s.get_traces().cpu().numpy(), s.get_step())


def _same(a, b):
    for x, y in zip(a, b):
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y)
        else:
            assert x == y


def _small_shots(n_shots=5, nt=80):
    return wl.shots_c3(nx=40, ny=34, nz=22, n_shots=n_shots, nt=nt, n_rec=6, seed=31)


@pytest.mark.parametrize("prec", PRECS)
def test_shots_in_one_solver_match_one_shot_solvers(prec):
    w = _small_shots()
    multi = _solver(w, prec)
    multi.step(w.nt)
    tr = multi.get_traces().cpu().numpy()
    u = multi.get_wavefield(0).cpu().numpy().reshape(w.n_shots, -1)
    assert tr.shape == (w.n_shots, len(w.rec_node), 3, w.nt)
    for k in range(w.n_shots):
        one = _solver(wl.single_shot(w, k), prec)
        one.step(w.nt)
        assert np.array_equal(one.get_traces().cpu().numpy()[0], tr[k]), k
        assert np.array_equal(one.get_wavefield(0).cpu().numpy(), u[k]), k
        one.close()
    # shot 2 against the oracle
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    w2 = wl.single_shot(w, 2)
    ref, _, _, _ = oasm.simulate(m, w.nt, w2.src_node, w2.src_comp, w2.wavelet, w2.rec_node)
    err = _rel(tr[2], ref)
    print("shot 2 %s traces vs oracle %.3e" % (prec, err))
    assert err <= TRACE_TOL


@pytest.mark.parametrize("prec", ["fp64", "int8"])
def test_grid_cap_strides_over_the_same_work(prec):
    w = _small_shots(n_shots=4, nt=40)
    a = _solver(w, prec, graph_steps=0)
    b = _solver(w, prec, persistent_groups=24, graph_steps=0)   # fewer work-groups than work items
    c = _solver(w, prec, persistent_groups=3, graph_steps=0)    # rounded up to 8
    for s in (a, b, c):
        s.step(w.nt)
    ref = _state(a)
    _same(_state(b), ref)
    _same(_state(c), ref)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n_shots", [1, 3])
def test_captured_graph_replays_match_direct_launches(prec, n_shots):
    import torch
    w = _small_shots(n_shots=n_shots, nt=120) if n_shots > 1 else wl.layered_c2(nx=30, ny=26, nz=20, nt=120, seed=32)
    direct = _solver(w, prec, graph_steps=0)
    graph = _solver(w, prec, graph_steps=8)
    # pieces: whole replays only, replays plus a tail, odd lengths (parity flips), short calls
    for n in (16, 20, 17, 3, 24, 9, 31):
        direct.step(n)
        graph.step(n)
        _same(_state(graph), _state(direct))
        # eager work between the replays
        x = torch.randn(1000, device="cuda", dtype=torch.float64)
        assert torch.isfinite((x * 2.0).sum()).item()
    assert graph.get_step() == 120


@pytest.mark.parametrize("prec", ["fp64", "int8"])
def test_uneven_batch_matches_individual_runs(prec):
    from paper_2404_13683_amd.ovfem import Batch
    doms = wl.uneven_domains_c3(n_domains=4, smallest=(10, 12, 9), largest=(40, 36, 24), nt=70, n_rec=4)
    shots = _small_shots(n_shots=3, nt=70)
    work = doms + [shots]
    alone = [_solver(d, prec) for d in work]
    members = [_solver(d, prec) for d in work]
    # members start from different step counters
    alone[1].step(5)
    members[1].step(5)
    batch = Batch(members)
    batch.step(30)
    batch.set_tuning(persistent_groups=16)
    batch.step(35)
    batch.close()
    for k, (a, m) in enumerate(zip(alone, members)):
        a.step(65)
        _same(_state(m), _state(a))
        assert m.get_step() == (70 if k == 1 else 65)


@pytest.mark.parametrize("prec", ["fp64", "int8"])
def test_uneven_batch_replayed_from_captured_graphs(prec):
    """Blocks of 12 batch steps replayed from a captured graph (step base in device memory),
    with eager reads between the calls, uneven call lengths that start off the block
    boundary, a member stepped alone in between (its tables are uploaded again), a grid cap
    switched on, and the graph switched off: bitwise the plain per-step launches."""
    from paper_2404_13683_amd.ovfem import Batch
    doms = wl.uneven_domains_c3(n_domains=3, smallest=(10, 12, 9), largest=(34, 30, 20), nt=140, n_rec=4, seed=12)
    shots = _small_shots(n_shots=2, nt=140)
    work = doms + [shots]
    plain = [_solver(d, prec) for d in work]
    graph = [_solver(d, prec) for d in work]
    bp, bg = Batch(plain), Batch(graph)
    bg.set_graph(12)
    for n in (5, 31, 24):
        bp.step(n)
        bg.step(n)
        _same(_state(graph[0]), _state(plain[0]))  # eager work between replays
    plain[2].step(3)
    graph[2].step(3)
    for b in (bp, bg):
        b.set_tuning(persistent_groups=16)
        b.step(40)
    bg.set_graph(0)
    bp.step(7)
    bg.step(7)
    for b in (bp, bg):
        b.close()
    for a, m in zip(plain, graph):
        _same(_state(m), _state(a))
    assert graph[2].get_step() == 110 and graph[0].get_step() == 107


def test_damped_batch_with_graph_steps_launches_plainly():
    """Damped batches are not captured: with graph steps set they step as plain launches,
    bitwise equal to their members stepped alone."""
    from paper_2404_13683_amd.ovfem import Batch
    doms = wl.uneven_domains_c3(n_domains=2, smallest=(10, 9, 8), largest=(21, 18, 12), nt=40, n_rec=3, seed=13)
    alone = [_solver(d, "int8") for d in doms]
    members = [_solver(d, "int8") for d in doms]
    for x in alone + members:
        x.set_damping(2.0, 1e-4 * doms[0].dt)
    b = Batch(members)
    b.set_graph(12)
    b.step(31)
    b.close()
    for a, m in zip(alone, members):
        a.step(31)
        _same(_state(m), _state(a))


def test_batch_rejects_mixed_precision():
    from paper_2404_13683_amd.ovfem import Batch, OvfemError
    d = wl.uneven_domains_c3(n_domains=2, smallest=(8, 8, 8), largest=(12, 10, 9), nt=10, n_rec=2)
    b = Batch([_solver(d[0], "fp64"), _solver(d[1], "int8")])
    with pytest.raises(OvfemError):
        b.step(1)


@pytest.mark.parametrize("prec", PRECS)
def test_chunk_depth(prec):
    """FP64: bitwise independent of the tiling.  INT8: within the trace bound of the oracle
    at every tiling (the exponents are per tile)."""
    w = wl.layered_c2(nx=33, ny=29, nz=40, nt=90, seed=33)
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    ref, _, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    got = {}
    for planes in (1, 7, 16, 41, 64):
        s = _solver(w, prec, chunk_planes=planes)
        s.step(w.nt)
        got[planes] = s.get_traces().cpu().numpy()[0]
        err = _rel(got[planes], ref)
        print("%s chunk %d: traces vs oracle %.3e" % (prec, planes, err))
        assert err <= TRACE_TOL
    if prec == "fp64":
        for planes in got:
            assert np.array_equal(got[planes], got[16])


@pytest.mark.parametrize("prec", PRECS)
def test_tile_rows(prec):
    """Tiles of 16 x 32 elements (512 threads) against the default 16 x 16: FP64 bitwise (the
    same element products and two-term node sums), INT8 within the trace bound of the oracle
    (its staging exponent spans the tile's staged block); ragged grids, matvec, and a damped
    run; a batch of members with 32-row tiles is bitwise its members stepped alone."""
    import torch

    from paper_2404_13683_amd.ovfem import Batch
    w = wl.layered_c2(nx=37, ny=70, nz=23, nt=80, seed=35)  # 71 node rows: 3 tiles of 31, 5 of 15
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    ref, _, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    u = torch.from_numpy(np.random.default_rng(3).standard_normal(3 * w.n_nodes)).cuda()
    ku_ref = oasm.matvec(u.cpu().numpy().reshape(m.node_shape), w.lam, w.mu, w.h).reshape(-1)
    out = {}
    for rows in (16, 32):
        s = _solver(w, prec, chunk_planes=9, tile_rows=rows)
        assert s.get_tuning()["tile_rows"] == rows
        s.step(w.nt)
        tr = s.get_traces().cpu().numpy()[0]
        ku = s.matvec(u).cpu().numpy()
        out[rows] = (tr, ku, s.get_wavefield(0).cpu().numpy())
        s.close()
        err, merr = _rel(tr, ref), _rel(ku, ku_ref)
        print("%s tile rows %d: traces vs oracle %.3e, matvec %.3e" % (prec, rows, err, merr))
        assert err <= TRACE_TOL and merr <= 1e-12
    if prec.startswith("fp64"):
        for a, b in zip(out[16], out[32]):
            assert np.array_equal(a, b)
    # damped, and a batch of 32-row members against stepping alone
    d1 = wl.layered_c2(nx=20, ny=40, nz=12, nt=40, seed=36)
    d2 = wl.layered_c2(nx=33, ny=17, nz=10, nt=40, seed=37)
    alone = [_solver(d, prec, tile_rows=32) for d in (d1, d2)]
    members = [_solver(d, prec, tile_rows=32) for d in (d1, d2)]
    for x in alone + members:
        x.set_damping(3.0, 2e-4 * d1.dt)
    b = Batch(members)
    b.step(40)
    b.close()
    for a, mm in zip(alone, members):
        a.step(40)
        _same(_state(mm), _state(a))


def test_batch_rejects_mixed_tile_rows():
    from paper_2404_13683_amd.ovfem import Batch, OvfemError
    d = wl.uneven_domains_c3(n_domains=2, smallest=(8, 8, 8), largest=(12, 10, 9), nt=10, n_rec=2)
    b = Batch([_solver(d[0], "fp64", tile_rows=16), _solver(d[1], "fp64", tile_rows=32)])
    with pytest.raises(OvfemError, match="tile rows"):
        b.step(1)


@pytest.mark.parametrize("n_shots", [1, 4])
def test_autotune_keeps_state_and_results(n_shots):
    w = _small_shots(n_shots=n_shots, nt=60) if n_shots > 1 else wl.layered_c2(nx=36, ny=30, nz=34, nt=60, seed=34)
    ref = _solver(w, "fp64")
    ref.step(w.nt)
    s = _solver(w, "fp64")
    s.step(25)
    before = _state(s)
    ms = s.autotune(steps=4)
    assert ms > 0.0
    _same(_state(s), before)
    t = s.get_tuning()
    assert t["chunk_planes"] in (8, 12, 16, 24, 32) and t["graph_steps"] in (0, 64)
    s.step(w.nt - 25)
    _same(_state(s), _state(ref))


def test_tuning_rejects_bad_values():
    from paper_2404_13683_amd.ovfem import OvfemError
    w = wl.homogeneous_c1(nx=6, ny=6, nz=6)
    s = _solver(w, "fp64")
    for bad in (dict(chunk_planes=0), dict(graph_steps=7), dict(graph_steps=-2), dict(persistent_groups=-1)):
        with pytest.raises(OvfemError):
            s.set_tuning(**bad)


@pytest.mark.parametrize("prec", PRECS)
def test_topography_removed_voxels_vs_oracle(prec):
    """Fractal free surface with air voxels removed over a nested basin, reduced size."""
    w = wl.topography_c5(nx=46, ny=38, nz=26, f0=60.0, nt=150)
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt, solid=w.solid)
    ref, u_ref, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    s = _solver(w, prec)
    s.step(w.nt)
    tr = s.get_traces().cpu().numpy()[0]
    u = s.get_wavefield(0).cpu().numpy().reshape(u_ref.shape)
    err_t, err_u = _rel(tr, ref), _rel(u, u_ref)
    print("topography %s traces %.3e wavefield %.3e" % (prec, err_t, err_u))
    assert err_t <= TRACE_TOL and err_u <= TRACE_TOL
    # nodes touching no solid voxel never move
    assert np.all(u[~w.touched_nodes()] == 0.0)
