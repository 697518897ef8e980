"""Benchmark of the fused OVFEM stepper on one MI355X.

Workload (one step = one pass of the whole hot path: gather, element products,
assembly and the central-difference update, with source injection and receivers):
three horizontal layers on 256 x 256 x 128 voxels (8.4 M elements, ~25 M free
DOF), h = 5 m, Vs 300/800/2000 m/s, Vp = 2 Vs, rho 1800/2100/2500 kg/m^3, seeded
+-10 % Gaussian-correlated (L = 50 m) lam/mu perturbation, Ricker 5 Hz, dt at
0.5 x CFL.  Inputs are synthetic and already resident in HBM when timing starts.

Both element-product paths run from reset for warmup + steps time steps: the
plain FP64 path and the INT8 matrix-core path.  `value` is the INT8 path's
DOF-updates per second; the FP64 path, their ratio and the INT8-vs-FP64 receiver
trace error are reported beside it.  The CPU oracle is timed on a bounded sample
of the same workload on the host's cores.

Other workloads (parity cases, one JSON line each, not the headline):
  --workload c3-shots    64 shots on 128 x 128 x 64 in one launch per step
  --workload c3-uneven   16 layered domains of uneven size, one batched launch per step
  --workload c5          512 x 512 x 256 fractal topography over a basin, air removed
  --workload c5-slab     512 x 512 x 32 of the same recipe: one GPU's share of c5 split 8 ways

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--workload NAME]
(--steps defaults to the workload's run length: 2000 for c2, 1000 for c3, 4000 for c5)
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


# run length of each workload: the trace comparison between the paths covers the whole run
# (in the first few hundred steps of the large models the receivers see only the scheme's
# numerical precursor, amplitudes far below any arrival, where relative errors mean little)
FULL_STEPS = {"c2": 2000, "c3-shots": 1000, "c3-uneven": 1000, "c5": 4000, "c5-slab": 4000}

KERNEL_SOURCES = ["paper_2404_13683_amd/csrc/kernels.hpp", "paper_2404_13683_amd/csrc/refmat.hpp"]
EQUAL_ACCURACY = os.path.join(ROOT, "tests", "golden", "equal_dispersion_accuracy.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "layer_kernel_counters_layered_256x256x128.txt")


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path_name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel factor)."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    kv = {}
    for line in open(COUNTERS_FILE):
        line = line.strip()
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha") != kernel_sha():
        return None
    try:
        f = float(kv["%s_fetch_kib" % path_name]) * float(kv["fetch_factor"])
        w = float(kv["%s_write_kib" % path_name]) * float(kv["write_factor"])
    except KeyError:
        return None
    return (f + w) * 1024.0


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


def profile_counters(path_name):
    """Busy fractions of the stepper kernel from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    kv = {}
    for line in open(COUNTERS_FILE):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha") != kernel_sha():
        return None
    out = {}
    for key in ("valu_busy", "mfma_busy", "waves_per_simd", "wait_frac"):
        if "%s_%s" % (path_name, key) in kv:
            out[key] = float(kv["%s_%s" % (path_name, key)])
    return out or None


def trace_errors(a, b):
    """a against the reference b, both [..., receiver, component, step]: the pooled relative
    L2, the largest per-channel relative L2 over channels whose norm is at least 1e-6 of the
    largest channel's, and the error measure of Sec. 3, Eq. (18) (mean over channels of
    sum_t (a - b)^2 / sum_t b^2, channels with a zero reference left out)."""
    a = np.asarray(a).reshape(-1, np.shape(a)[-1])
    b = np.asarray(b).reshape(-1, np.shape(b)[-1])
    pooled = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    cn = np.linalg.norm(b, axis=1)
    sel = cn >= 1e-6 * cn.max()
    per = float(np.max(np.linalg.norm((a - b)[sel], axis=1) / cn[sel]))
    nz = cn > 0
    err18 = float(np.mean(np.sum((a - b)[nz] ** 2, axis=1) / cn[nz] ** 2))
    return {"trace_rel_l2": pooled, "per_channel_max_rel_l2": per, "err_eq18": err18}


def algorithmic_bytes(nx, ny, nz, shots=1):
    """Bytes a step must move: per shot u^n, u^{n-1} read and u^{n+1} written (72 B per node);
    once, dt^2/m per node (8 B) and lam, mu per element (16 B)."""
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    return 72 * nodes * shots + 8 * nodes + 16 * nx * ny * nz


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


def time_path(wl, prec, warmup, steps, autotune=True, chunk_planes=0, stages=8, element="ovfem"):
    """One solver (all shots of the workload): ms per step and the traces."""
    from paper_2404_13683_amd.ovfem import Solver
    s = Solver.from_workload(wl, precision=prec, receivers_nt=warmup + steps, element=element)
    if prec == "int8":
        s.set_stages(stages)
    if chunk_planes:
        s.set_tuning(chunk_planes=chunk_planes)
    elif autotune:
        s.autotune(steps=20)
    tuning = s.get_tuning()
    s.reset()
    ms = _timed(s.step, warmup, steps)
    traces = s.get_traces().cpu().numpy()
    s.close()
    return ms, traces, tuning


def time_batch(wls, prec, warmup, steps):
    """A batch of solvers of uneven size stepped together."""
    from paper_2404_13683_amd.ovfem import Batch, Solver
    sols = [Solver.from_workload(w, precision=prec, receivers_nt=warmup + steps) for w in wls]
    b = Batch(sols)
    ms = _timed(b.step, warmup, steps)
    traces = np.concatenate([s.get_traces().cpu().numpy().reshape(-1, warmup + steps) for s in sols])
    b.close()
    for s in sols:
        s.close()
    return ms, traces, None


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
        return [w], ("topography-basin-512x512x256 (67M voxels, %d free DOF, air removed), h=2 m, dt=%.4e s"
                     % (w.free_dof(), w.dt)), False
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
                    help="timed steps (default: the workload's own run length, 2000 for c2, 1000 for "
                         "c3-shots and c3-uneven, 4000 for c5)")
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--paths", default="fp64,int8,fp64-sf")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3-shots", "c3-uneven", "c5", "c5-slab"])
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--chunk-planes", type=int, default=0, help="fixed z-chunk depth instead of autotuning")
    ap.add_argument("--no-equal-accuracy", action="store_true", help="skip the trilinear comparison")
    ap.add_argument("--stage-sweep", action="store_true",
                    help="also time the INT8 path with 4..7 digit stages (accuracy/speed trade, Table 3)")
    ap.add_argument("--copy-probe", type=int, default=0, help="only run a plain copy of this many bytes")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py: the stepper runs on one GPU (--gpus %d requested); it does not shard a "
              "model or its shots across GPUs" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.steps is None:
        args.steps = FULL_STEPS[args.workload]

    import torch

    torch.cuda.set_device(0)
    nt = args.warmup + args.steps
    wls, desc, batched = make_workload(args.workload, nt)
    free_dof = sum(w.free_dof() * w.n_shots for w in wls)
    n_elem = sum(w.nx * w.ny * w.nz * w.n_shots for w in wls)
    bytes_step = sum(algorithmic_bytes(w.nx, w.ny, w.nz, w.n_shots) for w in wls)
    paths = args.paths.split(",")
    res = {}
    for p in paths:
        if batched:
            ms, tr, tuning = time_batch(wls, p, args.warmup, args.steps)
        else:
            ms, tr, tuning = time_path(wls[0], p, args.warmup, args.steps, autotune=not args.no_autotune,
                                       chunk_planes=args.chunk_planes)
        res[p] = {"ms_per_step": ms, "value": free_dof / (ms * 1e-3), "traces": tr, "tuning": tuning}
        print("[bench] %s %s: %.4f ms/step, %.4e DOF-updates/s, tuning %s"
              % (args.workload, p, ms, res[p]["value"], tuning), file=sys.stderr, flush=True)
    head = "int8" if "int8" in res else paths[0]
    ms = res[head]["ms_per_step"]
    hbm = bytes_step / (ms * 1e-3)
    sha = kernel_sha()
    traffic = measured_traffic(head) if args.workload == "c2" else None
    out = {
        "metric": METRIC,
        "value": res[head]["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8-digits(i8-mfma,int32-acc,exact)+f64" if head == "int8" else
                 ("int8-digits(bf16-mfma,exact)+f64" if head == "int8-bf16" else "f64"),
        "data": "synthetic",
        "config": {"workload": desc, "path": head, "tuning": res[head]["tuning"],
                   "domains": [[w.nx, w.ny, w.nz, w.n_shots] for w in wls] if len(wls) > 1 else
                   [wls[0].nx, wls[0].ny, wls[0].nz, wls[0].n_shots]},
        "roofline": {"bound": "hbm", "achieved": hbm / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                     "frac": hbm / HBM_PEAK, "traffic": traffic, "kernel_sha": sha,
                     "algorithmic_bytes_per_step": bytes_step,
                     "mfma_frac_int8_peak": (INT8_OPS_PER_ELEMENT * n_elem / (ms * 1e-3)) / INT8_PEAK
                     if head.startswith("int8") else None},
    }
    if "fp64" in res:
        f = res["fp64"]
        out["fp64_path"] = {"ms_per_step": f["ms_per_step"], "value": f["value"],
                            "traffic": measured_traffic("fp64") if args.workload == "c2" else None,
                            "fp64_frac": FP64_FLOP_PER_ELEMENT * n_elem / (f["ms_per_step"] * 1e-3) / FP64_PEAK,
                            "hbm_frac": bytes_step / (f["ms_per_step"] * 1e-3) / HBM_PEAK,
                            "tuning": f["tuning"]}
    if "fp64-sf" in res:
        f = res["fp64-sf"]
        out["fp64_sf_path"] = {"ms_per_step": f["ms_per_step"], "value": f["value"],
                               "traffic": measured_traffic("fp64-sf") if args.workload == "c2" else None,
                               "hbm_frac": bytes_step / (f["ms_per_step"] * 1e-3) / HBM_PEAK, "tuning": f["tuning"],
                               "note": "the OVFEM product sum-factorised in FP64 (a stronger FP64 baseline than the "
                                       "dense form the paper compares against)"}
        if "fp64" in res:
            out["fp64_sf_path"]["trace_rel_l2_vs_fp64"] = float(
                np.linalg.norm(f["traces"] - res["fp64"]["traces"]) / np.linalg.norm(res["fp64"]["traces"]))
    if "fp64" in res and head != "fp64":
        out["int8_vs_fp64"] = {"speedup": res["fp64"]["ms_per_step"] / res[head]["ms_per_step"],
                               **trace_errors(res[head]["traces"], res["fp64"]["traces"]),
                               "steps_compared": nt}
    copy_bw = copy_bandwidth()
    out["roofline"]["copy_GBps"] = copy_bw / 1e9
    out["roofline"]["frac_of_copy"] = hbm / copy_bw
    out["roofline"]["counters"] = profile_counters(head) if args.workload == "c2" else None
    if head.startswith("int8"):
        out["roofline"]["limiter"] = ("not HBM: the element phase's instruction issue and dependency latency; "
                                      "timing-only copies of the kernel put the matrix-core digit products at "
                                      "29 % of the step, the node phase at 12 %, the FP64 recombination at 11 %")
    if args.stage_sweep and not batched and "fp64" in res:
        sweep = []
        for M in (4, 5, 6, 7):
            ms_m, tr_m, tun_m = time_path(wls[0], "int8", args.warmup, args.steps,
                                          autotune=not args.no_autotune, chunk_planes=args.chunk_planes, stages=M)
            b = res["fp64"]["traces"]
            sweep.append({"stages": M, "ms_per_step": ms_m, "value": free_dof / (ms_m * 1e-3),
                          "trace_rel_l2_vs_fp64": float(np.linalg.norm(tr_m - b) / np.linalg.norm(b)),
                          "tuning": tun_m})
            print("[bench] stages %d: %.4f ms/step" % (M, ms_m), file=sys.stderr, flush=True)
        out["stage_sweep"] = sweep
    if args.workload == "c2" and "int8" in res and not args.no_equal_accuracy:
        # Sec. 3's comparison with the trilinear element at equal accuracy: the trilinear
        # FP64 kernel on the same model, and the mesh refinement it needs for the same
        # numerical dispersion (oracle Bloch analysis, stored with the script that wrote it)
        ms_t, _, tun_t = time_path(wls[0], "fp64", args.warmup, args.steps, autotune=not args.no_autotune,
                                   chunk_planes=args.chunk_planes, element="trilinear")
        ms_ts, _, _ = time_path(wls[0], "fp64-sf", args.warmup, args.steps, autotune=not args.no_autotune,
                                chunk_planes=args.chunk_planes, element="trilinear")
        fx = json.load(open(EQUAL_ACCURACY))
        row = [r for r in fx["rows"] if r["ppw_ovfem"] == 10][0]
        out["equal_accuracy"] = {
            "trilinear_fp64_ms_per_step": ms_t, "trilinear_tuning": tun_t,
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
        out["cpu_baseline"] = cpu_baseline(wls[0], args.cpu_budget, label=desc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
