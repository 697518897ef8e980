"""GPU: ovfem_batch_step_noalloc (argument tables in the library's fixed device array)
against ovfem_batch_step (tables in buffers the library allocates).

Both run the same kernels on the same tables, so wavefields, traces and step counters must
agree bitwise.  Two calls in a row: a batch of uneven grids with a multi-shot member, then a
smaller batch (the second call's tables overwrite the first's in the shared array).  The
size limit and the "member not yet stepped" state are refused with an error.
"""
import numpy as np
import pytest

from paper_2404_13683_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _workloads(sizes, nt, seed):
    out = [wl.layered_c2(nx=nx, ny=ny, nz=nz, nt=nt, n_rec=4, seed=seed + i) for i, (nx, ny, nz) in enumerate(sizes)]
    return out


def _members(ws, prec, shots=None):
    from paper_2404_13683_amd.ovfem import Solver
    ms = [Solver.from_workload(w, precision=prec) for w in ws]
    if shots is not None:
        ms.append(Solver.from_workload(shots, precision=prec))
    for m in ms:
        m.step(0)  # builds each member's dt^2/m table
    return ms


def _state(ms):
    return [(m.get_wavefield(0).cpu().numpy(), m.get_wavefield(1).cpu().numpy(), m.get_traces().cpu().numpy(),
             m.get_step()) for m in ms]


def _run(ws, prec, shots, calls, noalloc):
    from paper_2404_13683_amd.ovfem import Batch
    ms = _members(ws, prec, shots)
    b = Batch(ms)
    for n in calls:
        if noalloc:
            b.step_noalloc(n)
        else:
            b.step(n)
    st = _state(ms)
    b.close()
    for m in ms:
        m.close()
    return st


def _assert_same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        for p, q in zip(x, y):
            if isinstance(p, np.ndarray):
                assert np.array_equal(p, q)
            else:
                assert p == q


@pytest.mark.parametrize("prec", ["int8", "fp64-sf"])
def test_noalloc_batch_step_matches_batch_step_on_two_calls(prec):
    shots = wl.shots_c3(nx=24, ny=20, nz=14, n_shots=3, nt=60, n_rec=4, seed=8)
    big = _workloads([(37, 23, 19), (16, 16, 16), (31, 9, 12)], nt=60, seed=40)
    # first call: three uneven grids and a 3-shot grid, advanced 23 + 14 steps
    a = _run(big, prec, shots, (23, 14), noalloc=False)
    b = _run(big, prec, shots, (23, 14), noalloc=True)
    _assert_same(a, b)
    # second call, smaller: two grids, 17 steps, after the larger tables were written
    small = _workloads([(12, 10, 9), (20, 6, 7)], nt=60, seed=70)
    a = _run(small, prec, None, (17,), noalloc=False)
    b = _run(small, prec, None, (17,), noalloc=True)
    _assert_same(a, b)
    assert b[0][3] == 17


def test_noalloc_batch_step_refuses_what_it_cannot_hold():
    from paper_2404_13683_amd.ovfem import Batch, OvfemError, Solver
    w = wl.layered_c2(nx=6, ny=5, nz=4, nt=8, n_rec=2, seed=3)
    m = Solver.from_workload(w, precision="int8")
    b = Batch([m])
    with pytest.raises(OvfemError, match="stepped|step it once"):
        b.step_noalloc(1)  # the member's dt^2/m table is not built yet
    m.step(0)
    b.step_noalloc(2)
    assert m.get_step() == 2
    b.close()
    m.close()
    many = wl.shots_c3(nx=40, ny=40, nz=4, n_shots=800, nt=4, n_rec=1, seed=9)  # 800 units > 702
    s = Solver.from_workload(many, precision="fp64")
    s.step(0)
    b = Batch([s])
    with pytest.raises(OvfemError, match="fixed array holds"):
        b.step_noalloc(1)
    assert s.get_step() == 0
    b.close()
    s.close()
