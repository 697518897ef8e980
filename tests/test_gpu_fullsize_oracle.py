"""GPU against full-length oracle runs at full size.

The references were written by tests/golden/make_fullsize_oracle.py, which steps the FP64
oracle over the whole run on the host (tens of minutes per case):
  * two shots of the 64-shot 128 x 128 x 64 workload, 1000 steps: receiver traces at every
    10th step, against all 64 shots advanced in one launch per step on each path.
Target: 1e-9 relative L2 over the stored samples.
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
    assert len(fixtures) >= 2
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
