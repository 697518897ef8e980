"""GPU: solvers on non-default streams, and two solvers running concurrently.

The library enqueues every kernel and copy of a solver on the stream it was created
with.  Runs on side streams (two solvers interleaved, each on its own stream) must give
bitwise the results of the same runs alone on the default stream.
"""
import numpy as np
import pytest

from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(w, prec, stream=None):
    """A solver for w created on `stream` (torch's current stream if None)."""
    import torch

    from paper_2404_13683_amd.ovfem import Solver
    with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
        return Solver.from_workload(w, precision=prec)


@pytest.mark.parametrize("prec", ["int8", "fp64-sf"])
def test_side_streams_and_concurrent_solvers_are_bitwise(prec):
    import torch
    a = wl.layered_c2(nx=40, ny=36, nz=24, f0=30.0, nt=150, seed=71)
    b = wl.shots_c3(nx=32, ny=30, nz=20, n_shots=3, f0=30.0, nt=150, n_rec=4, seed=72)
    ref = {}
    for name, w in (("a", a), ("b", b)):
        s = _run(w, prec)
        s.step(w.nt)
        ref[name] = (s.get_traces().cpu().numpy(), s.get_wavefield(0).cpu().numpy())
        s.close()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    xa, xb = _run(a, prec, sa), _run(b, prec, sb)
    for _ in range(5):  # interleaved: both streams busy at once
        with torch.cuda.stream(sa):
            xa.step(a.nt // 5)
        with torch.cuda.stream(sb):
            xb.step(b.nt // 5)
    for name, x in (("a", xa), ("b", xb)):
        # read back from the default stream: the binding orders it after the solver's stream
        tr, u = x.get_traces().cpu().numpy(), x.get_wavefield(0).cpu().numpy()
        assert np.array_equal(tr, ref[name][0]), name
        assert np.array_equal(u, ref[name][1]), name
        x.close()
