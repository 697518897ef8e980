"""GPU: the INT8 forms' accuracy contract, checked entry by entry against the oracle.

The paper scales each element by its own s_e before the integer split (Sec. 2, Eq. (10)) and
states that 8 digit stages are at least as accurate as FP64 (Sec. 3, Table 3).  The kernels
scale by a power of two shared by the nodes a work-group stages for one element layer, so
the contract is stated per entry against that block:

  * the owner work-group of node n (tile T of 15 x 15 node columns, x0 = 15 tx, y0 = 15 ty)
    computes n's element contributions of layer kk (kk = k-1, k) from the staged block of
    nodes x0-1..x0+15, y0-1..y0+15, planes kk and kk+1 (0 outside the grid);
  * its staging exponent S(T, kk) is max(-900, e) rounded up to a multiple of 4, e the
    exponent with 2^(e-1) <= m < 2^e for the block's largest magnitude m (S = -900 when the
    block is all zero);
  * every staged value v becomes q 2^(S-QB), q = rint(v 2^(QB-S)), QB = 8M - 2, an error of
    at most 2^(S-QB-1); the integer digit products are exact; the rest is FP64.

Hence, for every node n and component c,
    |(K u)_int8 - (K u)| <= sum over layers kk and the 4 elements e of layer kk at n of
                                h (lam_e r_lam + mu_e r_mu) 2^(S(T(n), kk) - QB - 1)
                            + 64 2^-53 sum_e h (lam_e |K_lam| + mu_e |K_mu|) |u_e|,
with r_lam, r_mu the largest row sums of |K_lam|, |K_mu|; the last term covers the FP64
rounding of both the kernels and the oracle.  The fields are chosen so that most entries are
far below their block's maximum: an early-time wavefield whose front decays steeply, node
magnitudes spread over 1e-30..1e30, and values near the exponent floor.
"""
import numpy as np
import pytest

from oracle import assembly as oasm
from oracle import element as oel
from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu

TN = 15          # owned node columns per tile side
EXP_FLOOR = -900
EXP_QUANT = 4
SLACK = 64 * 2.0 ** -53


def _staging_exponents(u, nx, ny, nz):
    """S[kk, ty, tx] for element layers kk = 0..nz-1 (formula in the module docstring)."""
    a = np.abs(u).max(axis=-1)  # (nz+1, ny+1, nx+1)
    tx_n, ty_n = nx // TN + 1, ny // TN + 1
    pad = np.zeros((nz + 1, TN * ty_n + 2, TN * tx_n + 2))
    pad[:, 1:ny + 2, 1:nx + 2] = a
    pm = np.zeros((nz + 1, ty_n, tx_n))
    for ty in range(ty_n):
        for tx in range(tx_n):
            pm[:, ty, tx] = pad[:, TN * ty:TN * ty + TN + 2, TN * tx:TN * tx + TN + 2].max(axis=(1, 2))
    m = np.maximum(pm[:-1], pm[1:])
    e = np.frexp(m)[1]
    S = np.where(m > 0, np.maximum(e, EXP_FLOOR), EXP_FLOOR)
    return -((-S) // EXP_QUANT) * EXP_QUANT


def contract_bound(u, lam, mu, h, M):
    """The per-entry bound of the module docstring, (nz+1, ny+1, nx+1, 3)."""
    QB = 8 * M - 2
    nz, ny, nx = lam.shape
    Kl, Km = oel.ovfem_reference()
    r_lam, r_mu = np.abs(Kl).sum(axis=1).max(), np.abs(Km).sum(axis=1).max()
    S = _staging_exponents(u, nx, ny, nz)
    w = h * (lam * r_lam + mu * r_mu)  # per element
    bound = np.zeros(u.shape[:3])
    jt = np.minimum(np.arange(ny + 1) // TN, S.shape[1] - 1)
    it = np.minimum(np.arange(nx + 1) // TN, S.shape[2] - 1)
    for kk in range(nz):
        # sum of w over the 4 elements of layer kk around each node of a plane
        p = np.zeros((ny + 2, nx + 2))
        p[1:ny + 1, 1:nx + 1] = w[kk]
        box = p[1:, 1:] + p[:-1, 1:] + p[1:, :-1] + p[:-1, :-1]  # (ny+1, nx+1)
        scale = np.ldexp(1.0, S[kk][jt[:, None], it[None, :]] - QB - 1)
        bound[kk] += box * scale      # plane kk: bottom corners of layer kk
        bound[kk + 1] += box * scale  # plane kk+1: top corners of layer kk
    absku = oasm.matvec(np.abs(u), lam, mu, h, K=(np.abs(Kl), np.abs(Km)))
    return bound[..., None] + SLACK * absku, absku


def _gpu_matvec(w, prec, u, stages=8, chunk_planes=None):
    import torch

    from paper_2404_13683_amd.ovfem import Solver
    s = Solver.from_workload(w, precision=prec)
    if prec == "int8":
        s.set_stages(stages)
    if chunk_planes:
        s.set_tuning(chunk_planes=chunk_planes)
    out = s.matvec(torch.from_numpy(np.ascontiguousarray(u).reshape(-1)).cuda()).cpu().numpy().reshape(u.shape)
    s.close()
    return out


def _early_wavefield():
    """C2's recipe at 64 x 48 x 32 after 24 oracle steps: a front that decays by hundreds of
    orders of magnitude across the domain (the scheme's numerical precursor)."""
    w = wl.layered_c2(nx=64, ny=48, nz=32, nt=24)
    m = oasm.Model(w.lam, w.mu, w.rho, w.h, w.fixed, w.dt)
    _, u, _, _ = oasm.simulate(m, w.nt, w.src_node, w.src_comp, w.wavelet, w.rec_node)
    return w, u


def _fields():
    w, u_early = _early_wavefield()
    rng = np.random.default_rng(11)
    shape = u_early.shape
    wide = rng.standard_normal(shape) * 10.0 ** rng.uniform(-30, 30, shape[:3])[..., None]
    tiny = rng.standard_normal(shape) * 10.0 ** rng.uniform(-300, -270, shape[:3])[..., None]
    tiny[:, :, : shape[2] // 2] = 0.0
    return w, {"early-wavefield": u_early, "magnitudes-1e+-30": wide, "near-exponent-floor": tiny}


@pytest.fixture(scope="module")
def fields():
    return _fields()


@pytest.mark.parametrize("prec,stages", [("int8", 8), ("int8", 6), ("int8-bf16", 8)])
def test_int8_matvec_meets_the_staging_exponent_bound_entry_by_entry(fields, prec, stages):
    w, cases = fields
    for name, u in cases.items():
        got = _gpu_matvec(w, prec, u, stages=stages)
        ref = oasm.matvec(u, w.lam, w.mu, w.h)
        bound, absku = contract_bound(u, w.lam, w.mu, w.h, stages)
        err = np.abs(got - ref)
        ratio = err / bound
        worst = np.unravel_index(np.argmax(ratio), ratio.shape)
        print("%s M=%d %s: max err/bound %.3f at %s (err %.3e, bound %.3e, |Ku| %.3e); median %.2e"
              % (prec, stages, name, ratio[worst], worst, err[worst], bound[worst], abs(ref[worst]),
                 np.median(ratio)))
        assert np.all(err <= bound)
        if stages == 8:
            # what the bound means for M = 8: the whole product at FP64 accuracy, and every
            # entry within six orders of magnitude of the largest to 1e-10 of its own scale
            assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
            big = absku >= 1e-6 * absku.max()
            assert np.all(err[big] <= 1e-10 * absku[big])


def test_int8_matvec_does_not_depend_on_the_chunk_depth(fields):
    """The staging exponent is a function of the layer's staged block only, so INT8 results
    are bitwise the same for every z-chunk depth (the FP64 paths already are)."""
    w, cases = fields
    for name, u in cases.items():
        ref = _gpu_matvec(w, "int8", u, chunk_planes=32)
        for planes in (5, 8, 16):
            got = _gpu_matvec(w, "int8", u, chunk_planes=planes)
            assert np.array_equal(got, ref), (name, planes)


def test_int8_steps_do_not_depend_on_the_chunk_depth():
    import torch

    from paper_2404_13683_amd.ovfem import Solver
    w = wl.layered_c2(nx=40, ny=33, nz=30, nt=60)
    out = []
    for planes in (7, 16, 31):
        s = Solver.from_workload(w, precision="int8")
        s.set_tuning(chunk_planes=planes)
        s.step(w.nt)
        out.append((s.get_traces().cpu().numpy(), s.get_wavefield(0).cpu().numpy()))
        s.close()
    for tr, u in out[1:]:
        assert np.array_equal(tr, out[0][0]) and np.array_equal(u, out[0][1])
    assert torch.cuda.is_available()
