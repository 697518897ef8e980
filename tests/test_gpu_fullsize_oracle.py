"""GPU against full-length oracle runs at full size.

The references were written by tests/golden/make_fullsize_oracle.py, which steps the FP64
oracle over the whole run on the host (tens of minutes per case):
  * four shots of the 64-shot 128 x 128 x 64 workload, 1000 steps: receiver traces at every
    10th step, against all 64 shots advanced in one launch per step on each path;
  * the layered 256 x 256 x 128 workload, 2000 steps: receiver traces at every 20th step;
  * the 96^3 adjoint workload, 1000 steps, checkpoints every 50: the misfit J and the
    discrete-adjoint gradient at 50 seeded voxels, against the GPU adjoint on each path.
Targets: 1e-9 relative on traces and gradients (relative L2 over the stored samples).
"""
import glob
import json
import os
import re

import numpy as np
import pytest

from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-9
PATHS = ("int8", "fp64", "fp64-sf")


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def _c3_fixtures():
    out = []
    for f in sorted(glob.glob(os.path.join(GOLDEN, "fullsize_c3_shot*.json"))):
        shot = int(re.search(r"shot(\d+)\.json$", f).group(1))
        out.append((shot, json.load(open(f))))
    return out


@pytest.mark.timeout(600)
def test_c3_shots_against_full_length_oracle_runs():
    from paper_2404_13683_amd.ovfem import Solver
    fixtures = _c3_fixtures()
    assert len(fixtures) >= 4
    w = wl.shots_c3()
    for shot, fx in fixtures:
        assert fx["nt"] == w.nt and fx["rec_node"] == [int(r) for r in w.rec_node]
    for prec in PATHS:
        s = Solver.from_workload(w, precision=prec)
        s.autotune(steps=4)
        s.reset()
        s.step(w.nt)
        tr = s.get_traces().cpu().numpy()
        s.close()
        for shot, fx in fixtures:
            err = _rel(tr[shot][..., fx["steps"]], np.array(fx["traces"]))
            print("c3 shot %d %s vs the oracle over %d steps: rel L2 %.3e" % (shot, prec, w.nt, err))
            assert err <= TOL


@pytest.mark.timeout(600)
def test_c2_against_the_full_length_oracle_run():
    """The layered 256 x 256 x 128 model over its whole 2000 steps on every path, against the
    oracle's own 2000-step run (receiver traces at every 20th step)."""
    from paper_2404_13683_amd.ovfem import Solver
    fx = json.load(open(os.path.join(GOLDEN, "fullsize_c2.json")))
    w = wl.layered_c2()
    assert fx["nt"] == w.nt and fx["rec_node"] == [int(r) for r in w.rec_node]
    assert (fx["nx"], fx["ny"], fx["nz"]) == (w.nx, w.ny, w.nz) and fx["dt"] == w.dt
    ref = np.array(fx["traces"])
    for prec in PATHS:
        s = Solver.from_workload(w, precision=prec)
        s.autotune(steps=4)
        s.reset()
        s.step(w.nt)
        tr = s.get_traces().cpu().numpy()[0]
        s.close()
        err = _rel(tr[..., fx["steps"]], ref)
        print("c2 %s vs the oracle over %d steps: rel L2 %.3e" % (prec, w.nt, err))
        assert err <= TOL


@pytest.mark.timeout(900)
def test_c4_adjoint_against_the_full_length_oracle_adjoint():
    import torch

    from paper_2404_13683_amd.ovfem import Solver
    fx = json.load(open(os.path.join(GOLDEN, "fullsize_c4.json")))
    true, start = wl.adjoint_c4()
    assert fx["nt"] == start.nt
    s = Solver.from_workload(true, precision="fp64")
    s.step(true.nt)
    d_obs = s.get_traces().clone()
    s.close()
    vox = tuple(np.array(fx["voxels"]).T)
    for prec in PATHS:
        s = Solver.from_workload(start, precision=prec)
        s.set_checkpointing(fx["ckpt_every"], start.nt)
        s.step(start.nt)
        res = (s.get_traces() - d_obs).contiguous()
        J = 0.5 * float(torch.sum(res * res))
        g_lam, g_mu = (g.cpu().numpy() for g in s.adjoint(res))
        s.close()
        eJ = abs(J - fx["J"]) / fx["J"]
        el_, em_ = _rel(g_lam[vox], fx["g_lam"]), _rel(g_mu[vox], fx["g_mu"])
        print("c4 %s vs the oracle: J %.3e, g_lam %.3e, g_mu %.3e (at %d voxels)" % (prec, eJ, el_, em_, len(vox[0])))
        assert eJ <= TOL and el_ <= TOL and em_ <= TOL
        # the sampled voxels carry the gradient's scale
        assert np.abs(g_lam[vox]).max() >= 1e-2 * fx["max_abs_g_lam"]
