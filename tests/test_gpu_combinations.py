"""GPU: the kernel combinations the other tests leave out.

Every stepper kernel is instantiated per (path, digit stage count, element) and per
damped/undamped step; these runs cover the damped kernels of the stage counts 4..7 and of
the trilinear element on every path, batches of trilinear solvers, and the adjoint with
6 digit stages and of the damped trilinear recursion, against the oracle's (damped)
stepper and adjoint or against stepping alone; a run whose precision and stage count
change between steps; and the batch kernels of every stage count against stepping alone.
"""
import numpy as np
import pytest

from oracle import assembly as oasm
from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _damped_case(seed=81, nt=200, element="ovfem"):
    w = wl.layered_c2(nx=26, ny=22, nz=18, f0=30.0, nt=nt, seed=seed)
    f0 = w.meta.get("f0", 30.0)
    alpha, beta = oasm.rayleigh_coefficients(0.02, 0.8 * f0, 1.25 * f0)
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt, alpha=alpha, beta=beta, element=element)
    ref, u_ref, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    return w, alpha, beta, ref, u_ref


def _solver(w, prec, alpha, beta, element="ovfem", stages=None):
    from paper_2404_13683_amd.ovfem import Solver
    s = Solver(w.nx, w.ny, w.nz, w.h, precision=prec)
    if element != "ovfem":
        s.set_element(element)
    if stages is not None:
        s.set_stages(stages)
    s.set_model(w.lam, w.mu, w.rho, w.solid)
    s.set_fixed_nodes(w.fixed)
    s.set_damping(alpha, beta)
    s.set_dt(w.dt)
    s.set_sources(w.src_node, w.src_comp, w.wavelet)
    s.set_receivers(w.rec_node, w.nt)
    return s


def test_damped_kernels_of_every_stage_count():
    """Damped runs with M = 4..8 digit stages: the error against the oracle's damped
    stepper falls with M as in the undamped case (M >= 6 within the 1e-9 trace bar)."""
    w, alpha, beta, ref, _ = _damped_case()
    err = {}
    for M in (4, 5, 6, 7, 8):
        s = _solver(w, "int8", alpha, beta, stages=M)
        s.step(w.nt)
        err[M] = _rel(s.get_traces().cpu().numpy()[0], ref)
        s.close()
    print("damped traces vs the oracle per stage count:", {k: "%.2e" % v for k, v in err.items()})
    for M in (6, 7, 8):
        assert err[M] <= 1e-9
    assert err[4] <= 1e-4 and err[5] <= 1e-6
    assert err[4] > err[5] > err[6]


@pytest.mark.parametrize("prec", ["fp64", "fp64-sf", "int8", "int8-bf16"])
def test_damped_trilinear_on_every_path(prec):
    w, alpha, beta, ref, u_ref = _damped_case(seed=82, element="trilinear")
    s = _solver(w, prec, alpha, beta, element="trilinear")
    s.step(w.nt)
    et = _rel(s.get_traces().cpu().numpy()[0], ref)
    eu = _rel(s.get_wavefield(0).cpu().numpy().reshape(u_ref.shape), u_ref)
    print("damped trilinear %s: traces %.3e wavefield %.3e" % (prec, et, eu))
    assert et <= 1e-9 and eu <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp64-sf", "int8"])
def test_trilinear_batch_is_stepping_alone(prec):
    from paper_2404_13683_amd.ovfem import Batch, Solver
    doms = wl.uneven_domains_c3(n_domains=3, smallest=(10, 12, 9), largest=(26, 22, 16), f0=60.0, nt=50, n_rec=3)

    def make(d):
        s = Solver.from_workload(d, precision=prec, element="trilinear")
        return s

    alone = [make(d) for d in doms]
    members = [make(d) for d in doms]
    b = Batch(members)
    b.step(50)
    b.close()
    for a, m in zip(alone, members):
        a.step(50)
        assert np.array_equal(a.get_traces().cpu().numpy(), m.get_traces().cpu().numpy())
        assert np.array_equal(a.get_wavefield(0).cpu().numpy(), m.get_wavefield(0).cpu().numpy())


def _adjoint_case(seed, element="ovfem", zeta=0.0):
    nx, ny, nz, nt = 12, 10, 9, 50
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = rng.uniform(1900, 2400, shape)
    vs = rng.uniform(500, 1100, shape)
    lam, mu = wl.lame_from_velocities(2.0 * vs, vs, rho)
    h = 4.0
    dt = wl.stable_dt(h, lam * 1.2, mu * 1.2, rho)
    f0 = 1.0 / (18 * dt)
    alpha, beta = oasm.rayleigh_coefficients(zeta, 0.8 * f0, 1.25 * f0) if zeta else (0.0, 0.0)
    src = np.array([wl.node_id(nx // 2, ny // 2, nz, nx, ny)], np.int64)
    rec = wl.surface_nodes(rng, 5, nx, ny, nz, exclude=src)
    w = wl.Workload("adjoint-combination", nx, ny, nz, h, lam, mu, rho, wl.box_fixed(nx, ny, nz), dt, nt, src,
                    np.array([2], np.int32), np.array([0], np.int32), wl.ricker(nt, dt, f0)[None, :], rec)
    mt = oasm.Model(lam * (1 + 0.1 * rng.standard_normal(shape)), mu, rho, h, w.fixed, dt, alpha=alpha, beta=beta,
                    element=element)
    d_obs, *_ = oasm.simulate(mt, nt, src, w.src_comp, w.wavelet, rec)
    m = oasm.Model(lam, mu, rho, h, w.fixed, dt, alpha=alpha, beta=beta, element=element)
    _, gl, gm = oasm.adjoint_gradient(m, nt, src, w.src_comp, w.wavelet, rec, d_obs)
    return w, alpha, beta, d_obs, gl, gm


@pytest.mark.parametrize("case", ["int8-M6", "trilinear-damped-fp64-sf", "trilinear-damped-int8"])
def test_adjoint_combinations(case):
    """The adjoint with 6 digit stages, and of the damped trilinear recursion, against the
    oracle's discrete adjoint."""
    import torch
    if case == "int8-M6":
        w, alpha, beta, d_obs, gl, gm = _adjoint_case(83)
        s = _solver(w, "int8", alpha, beta, stages=6)
    else:
        prec = {"trilinear-damped-fp64-sf": "fp64-sf", "trilinear-damped-int8": "int8"}[case]
        w, alpha, beta, d_obs, gl, gm = _adjoint_case(84, element="trilinear", zeta=0.05)
        s = _solver(w, prec, alpha, beta, element="trilinear")
    s.set_checkpointing(7, w.nt)
    s.step(w.nt)
    res = (s.get_traces() - torch.from_numpy(d_obs).cuda()[None]).contiguous()
    g_lam, g_mu = (g.cpu().numpy() for g in s.adjoint(res))
    el_, em_ = _rel(g_lam, gl), _rel(g_mu, gm)
    print("adjoint %s: %.3e %.3e" % (case, el_, em_))
    assert el_ <= 1e-9 and em_ <= 1e-9


def test_precision_switches_mid_run():
    """The INT8 staging exponent comes from the values each step stages, and every path
    reads and writes the same wavefield buffers, so the precision (and the stage count) can
    change between steps: a run that switches fp64 -> int8 (M = 6) -> fp64-sf -> int8-bf16 ->
    int8 matches the oracle's run."""
    from paper_2404_13683_amd.ovfem import Solver
    w = wl.layered_c2(nx=24, ny=20, nz=16, f0=30.0, nt=200, seed=85)
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    ref, u_ref, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    s = Solver.from_workload(w, precision="fp64")
    for prec, stages, n in (("fp64", None, 40), ("int8", 6, 40), ("fp64-sf", None, 40), ("int8-bf16", None, 40),
                            ("int8", 8, 40)):
        if prec == "int8-bf16":
            s.set_stages(8)
        s.set_precision(prec)
        if stages is not None:
            s.set_stages(stages)
        s.step(n)
    et = _rel(s.get_traces().cpu().numpy()[0], ref)
    eu = _rel(s.get_wavefield(0).cpu().numpy().reshape(u_ref.shape), u_ref)
    print("precision switches: traces %.3e wavefield %.3e" % (et, eu))
    assert et <= 1e-9 and eu <= 1e-9


@pytest.mark.parametrize("stages,damped", [(4, False), (5, False), (6, False), (7, False), (6, True)])
def test_uneven_batch_per_stage_count(stages, damped):
    """The batch kernels of every stage count (and the damped one with 6 digits) step an
    uneven batch bitwise as each member steps alone."""
    from paper_2404_13683_amd.ovfem import Batch, Solver
    doms = wl.uneven_domains_c3(n_domains=3, smallest=(10, 12, 9), largest=(30, 26, 18), f0=60.0, nt=60, n_rec=3)

    def make(d):
        s = Solver.from_workload(d, precision="int8")
        s.set_stages(stages)
        if damped:
            s.set_damping(0.5, 0.05 * d.dt)
        return s

    alone = [make(d) for d in doms]
    members = [make(d) for d in doms]
    b = Batch(members)
    b.step(60)
    b.close()
    for a, m in zip(alone, members):
        a.step(60)
        assert np.array_equal(a.get_traces().cpu().numpy(), m.get_traces().cpu().numpy())
        assert np.array_equal(a.get_wavefield(0).cpu().numpy(), m.get_wavefield(0).cpu().numpy())
        assert np.array_equal(a.get_wavefield(1).cpu().numpy(), m.get_wavefield(1).cpu().numpy())
