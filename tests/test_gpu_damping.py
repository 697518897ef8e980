"""GPU: Rayleigh-damped stepping (C = alpha M + beta K) against the oracle's damped stepper.

The damped step stages w = u^n + (beta/dt)(u^n - u^{n-1}) for the K product and keeps a
third nodal vector; these tests cover every path and the state machinery around it
(shots, batches, resume, tuning) to the same bars as the undamped runs.
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


def _damping(w, zeta=0.05):
    """Rayleigh coefficients for ratio zeta at 0.8 and 1.25 times the source frequency."""
    f0 = w.meta.get("f0", 1.0 / (25 * w.dt))
    return oasm.rayleigh_coefficients(zeta, 0.8 * f0, 1.25 * f0)


def _solver(w, prec, alpha, beta, **tuning):
    from paper_2404_13683_amd.ovfem import Solver
    s = Solver(w.nx, w.ny, w.nz, w.h, precision=prec, n_shots=w.n_shots)
    s.set_model(w.lam, w.mu, w.rho, w.solid)
    s.set_fixed_nodes(w.fixed)
    s.set_damping(alpha, beta)
    s.set_dt(w.dt)
    s.set_sources(w.src_node, w.src_comp, w.wavelet, w.src_shot)
    s.set_receivers(w.rec_node, w.nt)
    if tuning:
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


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", ["both", "stiffness"])
def test_damped_traces_match_the_oracle(prec, kind):
    w = wl.layered_c2(nx=30, ny=26, nz=22, f0=25.0, nt=240, seed=41)
    alpha, beta = _damping(w, zeta=0.02)
    if kind == "stiffness":
        alpha = 0.0
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt, alpha=alpha, beta=beta)
    ref, u_ref, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    m0 = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    ref0, _, _, _ = oasm.simulate(m0, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    s = _solver(w, prec, alpha, beta)
    s.step(w.nt)
    tr = s.get_traces().cpu().numpy()[0]
    u = s.get_wavefield(0).cpu().numpy().reshape(u_ref.shape)
    et, eu = _rel(tr, ref), _rel(u, u_ref)
    print("damped (%s) %s: traces %.3e wavefield %.3e; damping changes the traces by %.2e"
          % (kind, prec, et, eu, _rel(ref, ref0)))
    assert et <= TRACE_TOL and eu <= TRACE_TOL
    assert _rel(ref, ref0) > 1e-3  # the damping is not negligible in this case


def test_zero_damping_is_the_undamped_step_bitwise():
    w = wl.layered_c2(nx=20, ny=18, nz=16, f0=25.0, nt=80, seed=42)
    a = _solver(w, "int8", 0.0, 0.0)
    from paper_2404_13683_amd.ovfem import Solver
    b = Solver.from_workload(w, precision="int8")
    a.step(w.nt)
    b.step(w.nt)
    _same(_state(a), _state(b))


@pytest.mark.parametrize("prec", ["fp64", "int8"])
def test_damped_shots_batch_resume_and_tuning_are_bitwise(prec):
    from paper_2404_13683_amd.ovfem import Batch
    shots = wl.shots_c3(nx=28, ny=24, nz=18, n_shots=3, f0=60.0, nt=90, n_rec=4, seed=43)
    alpha, beta = _damping(shots)
    multi = _solver(shots, prec, alpha, beta)
    multi.step(shots.nt)
    tr = multi.get_traces().cpu().numpy()
    for k in range(shots.n_shots):
        one = _solver(wl.single_shot(shots, k), prec, alpha, beta)
        one.step(shots.nt)
        assert np.array_equal(one.get_traces().cpu().numpy()[0], tr[k]), k
    # uneven batch (members at different step counts and phases) vs stepping alone
    doms = wl.uneven_domains_c3(n_domains=3, smallest=(10, 12, 9), largest=(26, 22, 16), f0=60.0, nt=60, n_rec=3)
    alone = [_solver(d, prec, alpha, beta) for d in doms]
    members = [_solver(d, prec, alpha, beta) for d in doms]
    alone[0].step(1)
    members[0].step(1)
    alone[2].step(2)
    members[2].step(2)
    b = Batch(members)
    b.step(17)
    b.step(20)
    b.close()
    for a, m in zip(alone, members):
        a.step(37)
        _same(_state(m), _state(a))
    # resume from a saved state and retiling keep the run bitwise
    w = doms[1]
    ref = _solver(w, prec, alpha, beta)
    ref.step(w.nt)
    s = _solver(w, prec, alpha, beta)
    s.step(25)
    un, unm1 = s.get_wavefield(0).clone(), s.get_wavefield(1).clone()
    s.reset()
    s.set_wavefield(un, unm1, step=25)
    before = _state(s)
    s.autotune(steps=4)
    _same(_state(s), before)
    s.set_tuning(chunk_planes=16, tile_rows=16)  # the tiling the reference ran with (INT8 digits follow it)
    s.step(w.nt - 25)
    got, want = _state(s), _state(ref)
    _same(got[:2], want[:2])
    assert np.array_equal(got[2][..., 25:], want[2][..., 25:])  # traces from the resumed step on
    assert got[3] == want[3]


def test_damping_validation():
    import torch

    from paper_2404_13683_amd.ovfem import Batch, OvfemError, Solver
    w = wl.homogeneous_c1(nx=8, ny=8, nz=8, nt=20)
    s = Solver.from_workload(w, precision="fp64")
    for bad in ((-1.0, 0.0), (0.0, -1e-6), (float("nan"), 0.0), (0.0, float("inf"))):
        with pytest.raises(OvfemError):
            s.set_damping(*bad)
    with pytest.raises(OvfemError):
        s.set_damping(0.0, 100.0 * w.dt)  # beta far above dt: the set dt becomes unstable
    s.set_damping(10.0, 0.1 * w.dt)
    s.set_checkpointing(5, 20)
    s.step(20)
    g_lam, g_mu = s.adjoint(torch.zeros(s.n_rec * 3 * s.rec_nt, dtype=torch.float64, device="cuda"))
    assert not g_lam.abs().sum().item() and not g_mu.abs().sum().item()  # zero residual, zero gradient
    u = Solver.from_workload(w, precision="fp64")
    b = Batch([s, u])
    with pytest.raises(OvfemError):
        b.step(1)  # damped and undamped members
    b.close()


def _adjoint_case(seed, nx=12, ny=10, nz=9, nt=60, zeta=0.05):
    """Heterogeneous box, source at the surface centre, 5 surface receivers, Rayleigh
    damping of ratio zeta across the wavelet's band; observations from a perturbed lam."""
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    rho = rng.uniform(1900, 2400, shape)
    vs = rng.uniform(500, 1100, shape)
    lam, mu = wl.lame_from_velocities(2.0 * vs, vs, rho)
    h = 4.0
    dt = wl.stable_dt(h, lam * 1.2, mu * 1.2, rho)
    f0 = 1.0 / (18 * dt)
    alpha, beta = oasm.rayleigh_coefficients(zeta, 0.8 * f0, 1.25 * f0)
    src = np.array([wl.node_id(nx // 2, ny // 2, nz, nx, ny)], np.int64)
    rec = wl.surface_nodes(rng, 5, nx, ny, nz, exclude=src)
    w = wl.Workload("damped-adjoint", nx, ny, nz, h, lam, mu, rho, wl.box_fixed(nx, ny, nz), dt, nt, src,
                    np.array([2], np.int32), np.array([0], np.int32), wl.ricker(nt, dt, f0)[None, :], rec)
    mt = oasm.Model(lam * (1 + 0.1 * rng.standard_normal(shape)), mu, rho, h, w.fixed, dt, alpha=alpha, beta=beta)
    d_obs, *_ = oasm.simulate(mt, nt, src, w.src_comp, w.wavelet, rec)
    return w, alpha, beta, d_obs


@pytest.mark.parametrize("prec", ["fp64", "int8", "fp64-sf"])
def test_damped_adjoint_matches_the_oracle(prec):
    """The adjoint of the damped recursion (checkpoint segments of 9 steps) against the
    oracle's damped adjoint, which central differences pin on the CPU."""
    import torch
    w, alpha, beta, d_obs = _adjoint_case(seed=45)
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt, alpha=alpha, beta=beta)
    _, gl_ref, gm_ref = oasm.adjoint_gradient(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node, d_obs)
    m0 = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    _, gl_und, _ = oasm.adjoint_gradient(m0, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node, d_obs)
    s = _solver(w, prec, alpha, beta)
    s.set_checkpointing(9, w.nt)
    s.step(w.nt)
    res = (s.get_traces() - torch.from_numpy(d_obs).cuda()[None]).contiguous()
    g_lam, g_mu = (g.cpu().numpy() for g in s.adjoint(res))
    el_, em_ = _rel(g_lam, gl_ref), _rel(g_mu, gm_ref)
    print("damped adjoint %s: %.3e %.3e (damping changes the gradient by %.2e)"
          % (prec, el_, em_, _rel(gl_ref, gl_und)))
    assert el_ <= TRACE_TOL and em_ <= TRACE_TOL
    assert _rel(gl_ref, gl_und) > 1e-3
    # every state kept (the forward run steps through its checkpoint store, three damped
    # states apart), in two calls: the same traces, final state and gradient, bitwise
    tr9, u9 = s.get_traces().cpu().numpy(), s.get_wavefield(0).cpu().numpy()
    s.set_checkpointing(1, w.nt)
    s.step(w.nt // 3)
    s.step(w.nt - w.nt // 3)
    assert np.array_equal(s.get_traces().cpu().numpy(), tr9)
    assert np.array_equal(s.get_wavefield(0).cpu().numpy(), u9)
    g1_lam, g1_mu = (g.cpu().numpy() for g in s.adjoint(res))
    assert np.array_equal(g1_lam, g_lam) and np.array_equal(g1_mu, g_mu)


def test_damped_autograd_and_central_differences():
    """torch.autograd through the damped stepper; the FP64 gradient against central
    differences of the GPU's own misfit at seeded voxels."""
    import torch

    from paper_2404_13683_amd import autograd
    w, alpha, beta, d_obs = _adjoint_case(seed=46)
    s = _solver(w, "int8", alpha, beta)
    lam = torch.from_numpy(w.lam).cuda().requires_grad_(True)
    mu = torch.from_numpy(w.mu).cuda().requires_grad_(True)
    tr = autograd.traces(s, lam, mu, w.rho, nt=w.nt, ckpt_every=13)
    J = 0.5 * ((tr[0] - torch.from_numpy(d_obs).cuda()) ** 2).sum()
    J.backward()
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt, alpha=alpha, beta=beta)
    _, gl_ref, gm_ref = oasm.adjoint_gradient(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node, d_obs)
    assert _rel(lam.grad.cpu().numpy(), gl_ref) <= TRACE_TOL
    assert _rel(mu.grad.cpu().numpy(), gm_ref) <= TRACE_TOL

    f = _solver(w, "fp64", alpha, beta)

    def J_of(la, m_):
        f.set_model(la, m_, w.rho)
        f.set_damping(alpha, beta)
        f.set_dt(w.dt)
        f.step(w.nt)
        r = (f.get_traces() - torch.from_numpy(d_obs).cuda()).cpu().numpy()
        return 0.5 * float(np.sum(r * r))

    rng = np.random.default_rng(47)
    g = lam.grad.cpu().numpy()
    cand = np.argwhere(np.abs(g) >= 1e-2 * np.abs(g).max())
    for idx in cand[rng.choice(len(cand), size=4, replace=False)]:
        k, j, i = map(int, idx)
        la = w.lam.copy()
        base = la[k, j, i]
        eps = 1e-3 * base
        la[k, j, i] = base + eps
        jp = J_of(la, w.mu)
        la[k, j, i] = base - eps
        jm = J_of(la, w.mu)
        fd = (jp - jm) / (2 * eps)
        print("damped FD lam %s: adjoint %.6e fd %.6e" % ((k, j, i), g[k, j, i], fd))
        assert abs(g[k, j, i] - fd) <= 1e-4 * abs(fd)
