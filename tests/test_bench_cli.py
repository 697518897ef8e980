"""Host-side checks of bench.py (no GPU): the one-GPU refusal, argument checks, and the
algorithmic byte count of the roofline."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + list(args), capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_zero_timed_steps_are_refused():
    r = _run("--steps", "0", "--no-cpu")
    assert r.returncode != 0
    assert "--steps must be at least 1" in (r.stderr + r.stdout)


def test_algorithmic_bytes_count_free_nodes_and_solid_voxels():
    """72 B per free node and shot (u^n, u^{n-1} read, u^{n+1} written), 8 B per free node
    (dt^2/m) and 16 B per solid voxel (lam, mu): counted here by brute force on a small
    topography model with removed voxels and fixed faces."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2404_13683_amd import workloads as wl
    w = wl.topography_c5(nx=20, ny=18, nz=12, nt=10)
    solid = w.solid.astype(bool)
    touched = np.zeros((w.nz + 1, w.ny + 1, w.nx + 1), bool)
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                touched[dz:dz + w.nz, dy:dy + w.ny, dx:dx + w.nx] |= solid
    fixed = np.asarray(w.fixed, bool).reshape(touched.shape)
    free = int(np.count_nonzero(touched & ~fixed))
    assert w.free_dof() == 3 * free
    assert bench.algorithmic_bytes(w) == 72 * free * w.n_shots + 8 * free + 16 * int(np.count_nonzero(solid))


def test_adjoint_shot_count_below_one_is_refused():
    r = _run("--workload", "c4-adjoint", "--adjoint-shots", "0")
    assert r.returncode != 0
    assert "--adjoint-shots must be at least 1" in (r.stderr + r.stdout)


def test_surface_shots_keep_shot_zero_and_move_the_source():
    """with_surface_shots: shot 0 is the workload's own source; the others are the same
    component and wavelet at distinct top-surface nodes that are not receivers."""
    sys.path.insert(0, ROOT)
    from paper_2404_13683_amd import workloads as wl
    _, w = wl.adjoint_c4(nx=12, ny=10, nz=8, nt=20, n_rec=6)
    m = wl.with_surface_shots(w, 4, seed=3)
    assert m.n_shots == 4 and list(m.src_shot) == [0, 1, 2, 3]
    assert m.src_node[0] == w.src_node[0] and np.array_equal(m.wavelet[0], w.wavelet[0])
    assert len(set(m.src_node.tolist())) == 4 and not set(m.src_node.tolist()) & set(w.rec_node.tolist())
    k = m.src_node[1:] // ((w.nx + 1) * (w.ny + 1))
    assert np.all(k == w.nz) and np.all(m.src_comp == w.src_comp[0])
    assert all(np.array_equal(m.wavelet[v], w.wavelet[0]) for v in range(4))
    assert np.array_equal(wl.single_shot(m, 0).src_node, w.src_node)
