"""Benchmark of the fused OVFEM stepper on one MI355X.

Workload (default; one step = one pass of the whole hot path: gather, element products,
assembly and the central-difference update, with source injection and receivers): the
512 x 512 x 256 voxel model (67 M voxels, h = 2 m) with seeded fractal surface topography
(+-40 m, air voxels removed) over a nested three-material basin (Vs 200/600/1500 m/s,
Vp = 2 Vs, rho 1800/2100/2500 kg/m^3), Ricker 5 Hz, dt at 0.5 x CFL, 4000 steps: the
largest single-GPU configuration of the method.  Inputs are synthetic and already
resident in HBM when timing starts.

Each element-product path (INT8 digit slices on the matrix cores, dense FP64 as the
paper evaluates it, sum-factorised FP64) first runs the workload's whole length from rest
(4000 steps for the default; its rate is `full_run_ms_per_step`), and the INT8-vs-FP64
receiver-trace error over that run is reported: the accuracy condition of the metric holds
for traces after all steps, whatever --steps is.  Then warmup + steps timed steps run from
the state halfway through that run, when the wave fills the model (a model still at rest
runs faster, from the clock the chip holds on zeros); `value` is the INT8 path's
DOF-updates per second over them.  The CPU oracle is timed on a bounded sample on the
host's cores.

Other workloads (parity cases, one JSON line each, not the headline):
  --workload c2          256 x 256 x 128, three layers with perturbations, 2000 steps
  --workload c3-shots    64 shots on 128 x 128 x 64 in one launch per step
  --workload c3-uneven   16 layered domains of uneven size, one batched launch per step
  --workload c5-slab     512 x 512 x 32 of the c5 recipe: one GPU's share of c5 split 8 ways
  --workload c4-adjoint  96^3 misfit gradient: forward run keeping every state on a tape in HBM
                         (or checkpoints every N steps, --ckpt-every N), then
                         the discrete adjoint (backward step + gradient terms) per path,
                         gradients checked against the stored full-length oracle adjoint

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--workload NAME]
(--steps defaults to the workload's run length: 4000 for c5, 2000 for c2, 1000 for c3)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s/step: INT8-MFMA vs FP64 path at ≤1e-9 trace rel err; % roofline"
HBM_PEAK = 8.0e12          # bytes/s
INT8_PEAK = 5.0e15         # dense INT8 MFMA ops/s
FP64_PEAK = 78.6e12        # FP64 vector flop/s
INT8_OPS_PER_ELEMENT = 2 * 48 * 24 * 8    # [AL; AM] (48 x 24) times 8 digit slices
FP64_FLOP_PER_ELEMENT = 2 * 2 * 24 * 24   # AL u and AM u in FP64


# run length of each workload: the untimed parity leg compares the paths' traces over it
FULL_STEPS = {"c2": 2000, "c3-shots": 1000, "c3-uneven": 1000, "c5": 4000, "c5-slab": 4000, "c4-adjoint": 1000}

KERNEL_SOURCES = ["paper_2404_13683_amd/csrc/kernels.hpp", "paper_2404_13683_amd/csrc/refmat.hpp"]
EQUAL_ACCURACY = os.path.join(ROOT, "tests", "golden", "equal_dispersion_accuracy.json")
C4_ORACLE = os.path.join(ROOT, "tests", "golden", "fullsize_c4.json")
# rocprofv3 counter summaries of the stepper kernels, per workload
COUNTERS_FILES = {
    "c2": os.path.join(ROOT, "profiles", "layer_kernel_counters_layered_256x256x128.txt"),
    "c5": os.path.join(ROOT, "profiles", "layer_kernel_counters_topography_512x512x256.txt"),
}


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def _counter_values(workload):
    """Key = value pairs of the workload's committed counter summary, if it was taken on the
    current kernel source (else None)."""
    f = COUNTERS_FILES.get(workload)
    if not f or not os.path.exists(f):
        return None
    kv = {}
    for line in open(f):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("kernel_sha") == kernel_sha() else None


def measured_traffic(workload, path_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if taken on the
    current kernel source: the bytes of the L2-to-memory read and write requests counted by
    size (32, 64, 128 B) when the summary has them, else FETCH_SIZE + WRITE_SIZE scaled by the
    copy-kernel factors."""
    kv = _counter_values(workload)
    if kv is None:
        return None
    try:
        if "%s_read_bytes" % path_name in kv:
            return float(kv["%s_read_bytes" % path_name]) + float(kv["%s_write_bytes" % path_name])
        f = float(kv["%s_fetch_kib" % path_name]) * float(kv["fetch_factor"])
        w = float(kv["%s_write_kib" % path_name]) * float(kv["write_factor"])
    except KeyError:
        return None
    return (f + w) * 1024.0


def traffic_config(workload, path_name):
    """The launch configuration the committed counters were taken at (chunk depth; 16-row
    tiles), so that `traffic` can be read beside the tuned configuration of the run."""
    kv = _counter_values(workload)
    if kv is None or "%s_chunk_planes" % path_name not in kv:
        return None
    return {"chunk_planes": int(float(kv["%s_chunk_planes" % path_name])), "tile_rows": 16}


def profile_counters(workload, path_name):
    """Busy fractions of the stepper kernel from the committed counter summary."""
    kv = _counter_values(workload)
    if kv is None:
        return None
    out = {}
    for key in ("valu_busy", "mfma_busy", "waves_per_simd", "wait_frac"):
        if "%s_%s" % (path_name, key) in kv:
            out[key] = float(kv["%s_%s" % (path_name, key)])
    return out or None


def limiter_text(frac_of_copy, counters):
    """What bounds the kernel, from the live bandwidth and the committed counters."""
    if frac_of_copy >= 0.8:
        return "HBM: %.0f %% of a plain copy's bandwidth" % (100 * frac_of_copy)
    if counters and "valu_busy" in counters:
        return ("instruction issue, not HBM (%.0f %% of a plain copy's bandwidth): VALU busy %.2f, "
                "MFMA busy %.2f, %.1f waves per SIMD (rocprofv3 counters)"
                % (100 * frac_of_copy, counters["valu_busy"], counters.get("mfma_busy", 0.0),
                   counters.get("waves_per_simd", 0.0)))
    return None


def copy_probe(nbytes):
    """A plain copy of a known size (float32 elementwise kernel: nbytes read, nbytes written),
    used to calibrate the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.add(src, 0.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}))


def data_probe(paths):
    """The stepper kernels on the 512 x 512 x 256 model from an all-zero wavefield and from a
    uniform random one (the same instructions; the staging exponent is the same in every
    layer of both), alternated twice, 30 steps each: ms per step from HIP events, for a
    counter pass that reads the clock as GRBM_GUI_ACTIVE cycles over the kernel time."""
    import torch

    from paper_2404_13683_amd import workloads
    from paper_2404_13683_amd.ovfem import Solver
    w = workloads.topography_c5(nt=400)
    n = 3 * w.n_nodes
    zero = torch.zeros(n, dtype=torch.float64, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    r1 = (torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5) * 1e-6
    r2 = (torch.rand(n, dtype=torch.float64, device="cuda", generator=g) - 0.5) * 1e-6
    out = {}
    for p in paths:
        s = Solver.from_workload(w, precision=p, receivers_nt=w.nt + 1)
        s.set_tuning(chunk_planes={"int8": 48, "fp64": 64}.get(p, 24))
        out[p] = []
        for name, (a, b) in (("zero", (zero, zero)), ("random", (r1, r2))) * 2:
            s.set_wavefield(a, b)
            out[p].append((name, _timed(s.step, 5, 25)))
        s.close()
    print(json.dumps({"data_probe_ms_per_step": out}))


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Bytes per second (read + written) of a plain device copy of nbytes: the bandwidth an
    HBM-bound kernel can reach on this GPU in practice."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    bw = 2.0 * src.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    return bw


def trace_errors(a, b):
    """a against the reference b, both [..., receiver, component, step]: the pooled relative
    L2, the largest per-channel relative L2 over channels whose norm is at least 1e-6 of the
    largest channel's, and the error measure of Sec. 3, Eq. (18) (mean over channels of
    sum_t (a - b)^2 / sum_t b^2, channels with a zero reference left out)."""
    a = np.asarray(a).reshape(-1, np.shape(a)[-1])
    b = np.asarray(b).reshape(-1, np.shape(b)[-1])
    nb = np.linalg.norm(b)
    if nb == 0.0:
        return {"trace_rel_l2": None, "per_channel_max_rel_l2": None, "err_eq18": None,
                "max_abs_diff": float(np.abs(a - b).max()), "note": "all reference traces are zero"}
    pooled = float(np.linalg.norm(a - b) / nb)
    cn = np.linalg.norm(b, axis=1)
    sel = cn >= 1e-6 * cn.max()
    per = float(np.max(np.linalg.norm((a - b)[sel], axis=1) / cn[sel]))
    nz = cn > 0
    err18 = float(np.mean(np.sum((a - b)[nz] ** 2, axis=1) / cn[nz] ** 2))
    return {"trace_rel_l2": pooled, "per_channel_max_rel_l2": per, "err_eq18": err18}


def algorithmic_bytes(w):
    """Bytes a step must move (free nodes and solid elements only): per free node and shot
    u^n, u^{n-1} read and u^{n+1} written (72 B); per free node dt^2/m (8 B); per solid
    element lam, mu (16 B)."""
    free_nodes = w.free_dof() // 3
    solid = w.n_elements if w.solid is None else int(np.count_nonzero(w.solid))
    return 72 * free_nodes * w.n_shots + 8 * free_nodes + 16 * solid


def _timed(step, warmup, steps):
    """HIP events on the current (= the solvers') stream around `steps` steps."""
    import torch
    step(warmup)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / max(steps, 1)


class PathRun:
    """The solvers of one element-product path for a workload (one solver with all shots,
    or a batch of uneven solvers), kept open between the timed and the full-length legs."""

    def __init__(self, wls, prec, rec_nt, batched, autotune=True, chunk_planes=0, stages=8, element="ovfem",
                 tile_rows=16):
        from paper_2404_13683_amd.ovfem import Batch, Solver
        self.solvers = [Solver.from_workload(w, precision=prec, receivers_nt=rec_nt, element=element)
                        for w in wls]
        self.batch = Batch(self.solvers) if batched else None
        for s in self.solvers:
            if prec == "int8":
                s.set_stages(stages)
            if not batched:
                if chunk_planes:
                    s.set_tuning(chunk_planes=chunk_planes, tile_rows=tile_rows)
                elif autotune:
                    s.autotune(steps=20)
        self.tuning = None if batched else self.solvers[0].get_tuning()

    def step(self, n):
        if self.batch is not None:
            self.batch.step(n)
        else:
            for s in self.solvers:
                s.step(n)

    def reset(self):
        for s in self.solvers:
            s.reset()

    def traces(self, nt):
        return np.concatenate([s.get_traces().cpu().numpy()[..., :nt].reshape(-1, nt) for s in self.solvers])

    def save_state(self):
        return [(s.get_step(), s.get_wavefield(0).clone(), s.get_wavefield(1).clone()) for s in self.solvers]

    def restore_state(self, state):
        for s, (n, un, unm1) in zip(self.solvers, state):
            s.set_wavefield(un, unm1, n)

    def close(self):
        if self.batch is not None:
            self.batch.close()
        for s in self.solvers:
            s.close()


def time_run(run, warmup, steps, state=None):
    """Time `steps` steps after `warmup` from rest, or from a saved state."""
    if state is None:
        run.reset()
    else:
        run.restore_state(state)
    return _timed(run.step, warmup, steps)


def full_run(run, full):
    """The workload's whole run from rest, timed (the rate a run sustains); returns the ms per
    step, the traces and the state halfway through, when the wavefield fills the model."""
    import torch
    run.reset()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run.step(full // 2)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    state = run.save_state()  # untimed
    torch.cuda.synchronize()
    e0.record(stream)
    run.step(full - full // 2)
    e1.record(stream)
    torch.cuda.synchronize()
    ms += e0.elapsed_time(e1)
    return ms / full, run.traces(full), state


def cpu_baseline(wl, budget_s=15.0, label=None):
    """The oracle stepping one shot of the same model on the host until the budget is spent."""
    from oracle import assembly as oasm
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = 1
    m = oasm.Model(wl.lam, wl.mu, wl.rho, wl.h, wl.fixed, wl.dt, solid=wl.solid)
    sel = np.asarray(wl.src_shot) == 0
    u = np.zeros(m.node_shape)
    up = np.zeros(m.node_shape)
    n = 0
    t0 = time.perf_counter()
    while True:
        F = oasm.forcing(m.node_shape, wl.src_node[sel], wl.src_comp[sel], wl.wavelet[sel, n % wl.wavelet.shape[1]])
        un = m.step(u, up, F)
        up, u = u, un
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    cpu = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    env = ", ".join("%s=%s" % (k, os.environ[k]) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")
                    if k in os.environ)
    return {"value": wl.free_dof() * n / dt, "unit": "DOF-updates/s", "cores": int(threads), "kind": "oracle",
            "sample": "%d full steps of one shot of %s (numpy FP64 oracle, %.1f s; %s, %d BLAS threads%s; "
                      "%d cores visible)" % (n, label or wl.name, dt, cpu, threads, "; " + env if env else "",
                                              len(os.sched_getaffinity(0)))}


def cpu_sample(name, wls):
    """(workload, label) the oracle is timed on: the first one-shot model of the workload, or,
    for the 512 x 512 x 256 model (whose host step would need ~50 GB of temporaries), the 32
    element layers just below its lowest air voxel (all solid, through the basin)."""
    import dataclasses

    from paper_2404_13683_amd import workloads
    w = wls[0]
    if name != "c5":
        return w, None
    kz = 32
    air_layers = np.nonzero((w.solid == 0).any(axis=(1, 2)))[0]
    k0 = max(0, (int(air_layers.min()) if air_layers.size else w.nz) - kz)

    def remap(nodes):
        out = []
        for nd in np.asarray(nodes, np.int64):
            i, j, k = nd % (w.nx + 1), (nd // (w.nx + 1)) % (w.ny + 1), nd // ((w.nx + 1) * (w.ny + 1))
            if k0 <= k <= k0 + kz:
                out.append(workloads.node_id(i, j, k - k0, w.nx, w.ny))
        return np.array(out, np.int64)

    # the model's source, moved to the top centre of the slab
    src = np.array([workloads.node_id(w.nx // 2, w.ny // 2, kz, w.nx, w.ny)], np.int64)
    layers = slice(k0, k0 + kz)
    slab = dataclasses.replace(w, nz=kz, lam=w.lam[layers], mu=w.mu[layers], rho=w.rho[layers],
                               solid=None if w.solid is None else w.solid[layers],
                               fixed=workloads.box_fixed(w.nx, w.ny, kz), src_node=src,
                               src_comp=w.src_comp[:len(src)], src_shot=w.src_shot[:len(src)],
                               wavelet=w.wavelet[:len(src)], rec_node=remap(w.rec_node))
    return slab, ("element layers %d..%d (all solid, through the basin) of the 512x512x256 topography model "
                  "(%d free DOF)" % (k0, k0 + kz - 1, slab.free_dof()))


def adjoint_bench(args):
    """The 96^3 misfit gradient on each path: the forward run from rest keeping every state
    (or with checkpoints every --ckpt-every steps), then the discrete adjoint, each timed
    with HIP events on the solver's stream; gradients at the stored voxels against the
    oracle's full-length adjoint."""
    import torch

    from paper_2404_13683_amd import workloads
    from paper_2404_13683_amd.ovfem import Solver
    fx = json.load(open(C4_ORACLE))
    true, start = workloads.adjoint_c4()
    shots = args.adjoint_shots
    if shots > 1:
        true, start = (workloads.with_surface_shots(w, shots) for w in (true, start))
    nt = start.nt
    if args.ckpt_every:
        every = args.ckpt_every
    else:
        # every state on the tape when (nt + 2) nodal vectors per shot take at most half the
        # free HBM (22 GB of 288 per shot for this model), else the stored oracle run's interval
        tape = (nt + 2) * shots * 3 * start.n_nodes * 8
        every = 1 if tape <= 0.5 * torch.cuda.mem_get_info()[0] else fx["ckpt_every"]
    s = Solver.from_workload(true, precision="fp64")
    s.step(nt)
    d_obs = s.get_traces().clone()
    s.close()
    vox = tuple(np.array(fx["voxels"]).T)
    stream = torch.cuda.current_stream()
    free_dof = start.free_dof() * shots
    out = {}
    for p in args.paths.split(","):
        s = Solver.from_workload(start, precision=p)
        if not args.no_autotune:
            s.autotune(steps=20)
        s.set_checkpointing(every, nt)
        s.reset()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(stream)
        s.step(nt)
        e1.record(stream)
        res = (s.get_traces() - d_obs).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g_lam, g_mu = s.adjoint(res)  # returns after its stream has drained
        e2.record(stream)
        torch.cuda.synchronize()
        adj_s = time.perf_counter() - t0
        fwd_ms = e0.elapsed_time(e1) / nt
        if shots > 1:
            # shot 0 is the stored oracle run's shot: its residual alone (the other shots'
            # set to zero) gives that run's misfit and gradient (untimed)
            res[1:] = 0.0
            g_lam, g_mu = s.adjoint(res)
        J = 0.5 * float(torch.sum(res * res))
        gl, gm = g_lam.cpu().numpy(), g_mu.cpu().numpy()
        rel = lambda a, b: float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
        out[p] = {"forward_ms_per_step": fwd_ms, "adjoint_ms_per_step": adj_s * 1e3 / nt,
                  "adjoint_value": free_dof * nt / adj_s, "tuning": s.get_tuning(),
                  "vs_oracle": {"J": abs(J - fx["J"]) / fx["J"], "g_lam": rel(gl[vox], fx["g_lam"]),
                                "g_mu": rel(gm[vox], fx["g_mu"]), "voxels": len(vox[0])}}
        print("[bench] c4-adjoint %s: forward %.4f ms/step, adjoint %.4f ms/step, vs oracle %s"
              % (p, fwd_ms, adj_s * 1e3 / nt, out[p]["vs_oracle"]), file=sys.stderr, flush=True)
        s.close()
    head = "int8" if "int8" in out else list(out)[0]
    line = {
        "metric": "adjoint gradient DOF-updates/s (backward step + gradient terms per step, and the forward "
                  "recompute when checkpoints are sparser than every step)",
        "value": out[head]["adjoint_value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": nt, "warmup": 0,
        "ms_per_step": out[head]["adjoint_ms_per_step"], "higher_is_better": True, "vs_baseline": None,
        "dtype": "int8-digits(i8-mfma,int32-acc,exact)+f64" if head == "int8" else "f64", "data": "synthetic",
        "config": {"workload": "adjoint 96^3 (%d free DOF%s), h=5 m, 1000 steps, %s, 32 surface receivers; start "
                              "model homogeneous against a +-15 %% smooth true model"
                              % (start.free_dof(), "" if shots == 1 else
                                 " per shot, %d shots in one solver (shot 0 at the surface centre, the others at "
                                 "seeded surface nodes; the misfit summed over the shots)" % shots,
                                 "every state kept (checkpoint tape)" if every == 1
                                 else "checkpoints every %d" % every), "path": head, "ckpt_every": every,
                   "shots": shots},
        "paths": out,
    }
    print(json.dumps(line))


def make_workload(name, nt):
    """(list of workloads, description, batched?) for a workload name."""
    from paper_2404_13683_amd import workloads
    if name == "c2":
        w = workloads.layered_c2(nt=nt)
        return [w], ("layered-256x256x128 (8.4M voxels, %d free DOF), h=5 m, Ricker 5 Hz, dt=%.4e s"
                     % (w.free_dof(), w.dt)), False
    if name == "c3-shots":
        w = workloads.shots_c3(nt=nt)
        return [w], ("64 shots on layered-128x128x64 (%d free DOF per shot), h=5 m, one launch per step"
                     % w.free_dof()), False
    if name == "c3-uneven":
        ws = workloads.uneven_domains_c3(nt=nt)
        return ws, ("16 layered domains 32^3..160x160x80 (%d free DOF in all), one batched launch per step"
                    % sum(w.free_dof() for w in ws)), True
    if name == "c5":
        w = workloads.topography_c5(nt=nt)
        return [w], ("topography-basin-512x512x256 (67M voxels, %d free DOF, air removed), h=2 m, Ricker 5 Hz, "
                     "dt=%.4e s" % (w.free_dof(), w.dt)), False
    if name == "c5-slab":
        # one GPU's share of the 512 x 512 x 256 model split eight ways along z
        w = workloads.topography_c5(nz=32, nt=nt)
        return [w], ("topography-basin slab 512x512x32 (one eighth of the 512x512x256 model along z, "
                     "%d free DOF), h=2 m, dt=%.4e s" % (w.free_dof(), w.dt)), False
    raise SystemExit("unknown workload %r" % name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's own run length, 4000 for c5, 2000 for c2, "
                         "1000 for c3-shots and c3-uneven)")
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--paths", default="fp64,int8,fp64-sf")
    ap.add_argument("--workload", default="c5",
                    choices=["c5", "c2", "c3-shots", "c3-uneven", "c5-slab", "c4-adjoint"])
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--chunk-planes", type=int, default=0, help="fixed z-chunk depth instead of autotuning")
    ap.add_argument("--tile-rows", type=int, default=16, choices=[16, 32],
                    help="tile height with --chunk-planes (element rows per work-group)")
    ap.add_argument("--no-equal-accuracy", action="store_true", help="skip the trilinear comparison")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the full-length run (trace comparison, sustained rate); the timed steps "
                         "then start from rest")
    ap.add_argument("--stage-sweep", action="store_true",
                    help="also time the INT8 path with 4..7 digit stages (accuracy/speed trade, Table 3)")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a plain copy of this many bytes")
    ap.add_argument("--data-probe", action="store_true",
                    help="only time the stepper kernels (--paths) on a zero and on a random wavefield")
    ap.add_argument("--adjoint-shots", type=int, default=1,
                    help="c4-adjoint: shots in the solver (shot 0 the stored oracle run's; its gradient alone "
                         "is checked against the oracle's)")
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="c4-adjoint: checkpoint interval (default: 1, every state on a tape in HBM and no "
                         "recompute, when it takes at most half the free memory; else 50)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.data_probe:
        import torch
        torch.cuda.set_device(0)
        data_probe(args.paths.split(","))
        return
    if args.gpus != 1:
        print("bench.py: the stepper runs on one GPU (--gpus %d requested); it does not shard a "
              "model or its shots across GPUs" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.adjoint_shots < 1:
        raise SystemExit("bench.py: --adjoint-shots must be at least 1")
    if args.workload == "c4-adjoint":
        import torch
        torch.cuda.set_device(0)
        adjoint_bench(args)
        return
    full = FULL_STEPS[args.workload]
    if args.steps is None:
        args.steps = full
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("bench.py: --steps must be at least 1 and --warmup at least 0")

    import torch

    torch.cuda.set_device(0)
    nt_timed = args.warmup + args.steps
    rec_nt = max(nt_timed, full)
    wls, desc, batched = make_workload(args.workload, rec_nt)
    free_dof = sum(w.free_dof() * w.n_shots for w in wls)
    # solid voxels (the useful element products; removed voxels are computed as zeros)
    n_elem = sum((w.n_elements if w.solid is None else int(np.count_nonzero(w.solid))) * w.n_shots for w in wls)
    bytes_step = sum(algorithmic_bytes(w) for w in wls)
    paths = args.paths.split(",")
    runs, res, tr, sustained, states = {}, {}, {}, {}, {}
    for p in paths:
        runs[p] = PathRun(wls, p, rec_nt, batched, autotune=not args.no_autotune, chunk_planes=args.chunk_planes,
                          tile_rows=args.tile_rows)
        state = None
        if not args.no_full_run:
            # the whole run from rest: traces for the parity comparison, the rate a run sustains,
            # and the state halfway through that the timed window starts from (an all-zero
            # wavefield runs 4-14 % faster than a filled one, from the clock the chip then holds)
            sustained[p], tr[p], state = full_run(runs[p], full)
            if p == "fp64":
                states[p] = state  # also the start of the stage sweep and the trilinear timings
            print("[bench] full run of %d steps on %s: %.4f ms/step" % (full, p, sustained[p]), file=sys.stderr,
                  flush=True)
        if state is not None:
            # the same steps once untimed: the first steps from a restored state in a process
            # ran 5-10 % slower than any later ones (measured on the 256 x 256 x 128 model)
            time_run(runs[p], args.warmup, min(args.steps, 50), state)
        ms = time_run(runs[p], args.warmup, args.steps, state)
        res[p] = {"ms_per_step": ms, "value": free_dof / (ms * 1e-3), "tuning": runs[p].tuning}
        if batched:
            # the batch's steps replayed from captured graphs of 24 steps, against plain launches
            runs[p].batch.set_graph(24)
            ms_g = time_run(runs[p], args.warmup, args.steps, state)
            res[p]["plain_ms_per_step"], res[p]["graph_ms_per_step"] = ms, ms_g
            if ms_g < ms:
                res[p].update(ms_per_step=ms_g, value=free_dof / (ms_g * 1e-3), tuning={"batch_graph_steps": 24})
            else:
                runs[p].batch.set_graph(0)
                res[p]["tuning"] = {"batch_graph_steps": 0}
            print("[bench] %s %s: batch plain %.4f ms/step, replayed graphs %.4f" % (args.workload, p, ms, ms_g),
                  file=sys.stderr, flush=True)
        print("[bench] %s %s: %.4f ms/step, %.4e DOF-updates/s, tuning %s"
              % (args.workload, p, ms, res[p]["value"], runs[p].tuning), file=sys.stderr, flush=True)
    head = "int8" if "int8" in res else paths[0]
    ms = res[head]["ms_per_step"]
    hbm = bytes_step / (ms * 1e-3)
    sha = kernel_sha()
    out = {
        "metric": METRIC,
        "value": res[head]["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "int8-digits(i8-mfma,int32-acc,exact)+f64" if head == "int8" else
                 ("int8-digits(bf16-mfma,exact)+f64" if head == "int8-bf16" else "f64"),
        "data": "synthetic",
        "config": {"workload": desc, "path": head, "tuning": res[head]["tuning"],
                   "batch_plain_vs_graph_ms": ({p: [res[p]["plain_ms_per_step"], res[p]["graph_ms_per_step"]]
                                                for p in res} if batched else None),
                   "domains": [[w.nx, w.ny, w.nz, w.n_shots] for w in wls] if len(wls) > 1 else
                   [wls[0].nx, wls[0].ny, wls[0].nz, wls[0].n_shots]},
        "roofline": {"bound": "hbm", "achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": hbm / HBM_PEAK, "traffic": measured_traffic(args.workload, head),
                     "traffic_config": traffic_config(args.workload, head), "kernel_sha": sha,
                     "algorithmic_bytes_per_launch": bytes_step,
                     "mfma_frac_int8_peak": (INT8_OPS_PER_ELEMENT * n_elem / (ms * 1e-3)) / INT8_PEAK
                     if head.startswith("int8") else None},
    }
    if "fp64" in res:
        f = res["fp64"]
        out["fp64_path"] = {"ms_per_step": f["ms_per_step"], "value": f["value"],
                            "traffic": measured_traffic(args.workload, "fp64"),
                            "fp64_frac": FP64_FLOP_PER_ELEMENT * n_elem / (f["ms_per_step"] * 1e-3) / FP64_PEAK,
                            "hbm_frac": bytes_step / (f["ms_per_step"] * 1e-3) / HBM_PEAK,
                            "tuning": f["tuning"]}
        if head != "fp64":
            out["int8_speedup_vs_fp64"] = f["ms_per_step"] / ms
    if "fp64-sf" in res:
        f = res["fp64-sf"]
        out["fp64_sf_path"] = {"ms_per_step": f["ms_per_step"], "value": f["value"],
                               "traffic": measured_traffic(args.workload, "fp64-sf"),
                               "hbm_frac": bytes_step / (f["ms_per_step"] * 1e-3) / HBM_PEAK, "tuning": f["tuning"],
                               "note": "the OVFEM product sum-factorised in FP64 (a stronger FP64 baseline than the "
                                       "dense form the paper compares against)"}
    if not args.no_full_run:
        out["timed_from_step"] = full // 2
        # the whole run from rest (not `value`)
        out["full_run_ms_per_step"] = sustained
    if not args.no_full_run and "fp64" in res:
        for p in paths:
            if p != "fp64":
                key = "int8_vs_fp64" if p == head else "%s_vs_fp64" % p.replace("-", "_")
                out[key] = dict(trace_errors(tr[p], tr["fp64"]), steps_compared=full,
                                run="every path from rest over the workload's %d steps" % full)
    for p in paths:
        runs[p].close()
    del runs
    if (not args.no_full_run and not batched and "int8" in res and "fp64" in res and not args.stage_sweep
            and args.workload in ("c5", "c2")):
        # the fewest digit stages that still meet the metric's accuracy condition (Table 3's
        # trade): 6 stages, 46 bits under the staging exponent, timed the same way
        r = PathRun(wls, "int8", rec_nt, batched, autotune=not args.no_autotune, chunk_planes=args.chunk_planes,
                    tile_rows=args.tile_rows, stages=6)
        sus6, tr6, st6 = full_run(r, full)
        time_run(r, args.warmup, min(args.steps, 50), st6)
        ms6 = time_run(r, args.warmup, args.steps, st6)
        out["int8_m6_path"] = {"stages": 6, "ms_per_step": ms6, "value": free_dof / (ms6 * 1e-3),
                               "full_run_ms_per_step": sus6, "tuning": r.tuning,
                               "vs_fp64": dict(trace_errors(tr6, tr["fp64"]), steps_compared=full)}
        r.close()
        del st6
        print("[bench] int8 with 6 digit stages: %.4f ms/step, traces vs FP64 %.2e"
              % (ms6, out["int8_m6_path"]["vs_fp64"]["trace_rel_l2"]), file=sys.stderr, flush=True)
    copy_bw = copy_bandwidth()
    out["roofline"]["copy_GBps"] = copy_bw / 1e9
    out["roofline"]["frac_of_copy"] = hbm / copy_bw
    counters = profile_counters(args.workload, head)
    out["roofline"]["counters"] = counters
    out["roofline"]["limiter"] = limiter_text(hbm / copy_bw, counters)
    if args.stage_sweep and "fp64" in res:
        sweep = []
        ref = PathRun(wls, "fp64", rec_nt, batched, autotune=not args.no_autotune, chunk_planes=args.chunk_planes)
        ref.reset()
        ref.step(full)
        b = ref.traces(full)
        ref.close()
        for M in (4, 5, 6, 7):
            r = PathRun(wls, "int8", rec_nt, batched, autotune=not args.no_autotune,
                        chunk_planes=args.chunk_planes, stages=M)
            ms_m = time_run(r, args.warmup, args.steps, states.get("fp64"))
            r.reset()
            r.step(full)
            tr_m = r.traces(full)
            r.close()
            sweep.append({"stages": M, "ms_per_step": ms_m, "value": free_dof / (ms_m * 1e-3),
                          "trace_rel_l2_vs_fp64": float(np.linalg.norm(tr_m - b) / np.linalg.norm(b)),
                          "tuning": r.tuning})
            print("[bench] stages %d: %.4f ms/step" % (M, ms_m), file=sys.stderr, flush=True)
        out["stage_sweep"] = sweep
    if not batched and "int8" in res and not args.no_equal_accuracy and args.workload in ("c2", "c5"):
        # Sec. 3's comparison with the trilinear element at equal accuracy: the trilinear
        # FP64 kernels on the same model, and the mesh refinement it needs for the same
        # numerical dispersion (oracle Bloch analysis, stored with the script that wrote it)
        tri = {}
        for p in ("fp64", "fp64-sf"):
            r = PathRun(wls, p, rec_nt, False, autotune=not args.no_autotune, chunk_planes=args.chunk_planes,
                        element="trilinear")
            # timed from the OVFEM run's halfway state, as the OVFEM paths are (the kernels'
            # instructions do not depend on the data; their clock does)
            tri[p] = (time_run(r, args.warmup, args.steps, states.get("fp64")), r.tuning)
            r.close()
        fx = json.load(open(EQUAL_ACCURACY))
        row = [r for r in fx["rows"] if r["ppw_ovfem"] == 10][0]
        ms_t, ms_ts = tri["fp64"][0], tri["fp64-sf"][0]
        out["equal_accuracy"] = {
            "trilinear_fp64_ms_per_step": ms_t, "trilinear_tuning": tri["fp64"][1],
            "trilinear_fp64_sf_ms_per_step": ms_ts,
            "dispersion_h_ratio": row["h_ratio"], "refinement_cost_factor": row["cost_factor"],
            "at": "10 points per S wavelength, RMS phase error %.2e" % row["rms_phase_error"],
            "speedup_vs_trilinear_fp64": row["cost_factor"] * ms_t / res["int8"]["ms_per_step"],
            "speedup_vs_trilinear_fp64_sf": row["cost_factor"] * ms_ts / res["int8"]["ms_per_step"],
            "sf_ovfem_vs_sf_trilinear": (row["cost_factor"] * ms_ts / res["fp64-sf"]["ms_per_step"]
                                         if "fp64-sf" in res else None),
            "context": "the paper reports 17.0x for INT8 OVFEM vs FP64 VFEM on an A100 (its own waveform error measure)"}
        print("[bench] trilinear fp64: %.4f ms/step, fp64-sf: %.4f ms/step" % (ms_t, ms_ts), file=sys.stderr,
              flush=True)
    if not args.no_cpu:
        sample, label = cpu_sample(args.workload, wls)
        out["cpu_baseline"] = cpu_baseline(sample, args.cpu_budget, label=label)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
