"""ctypes binding of libovfem (include/ovfem.h): argument marshalling only.

Every step of the computation runs in the HIP library.  Host-side inputs (model,
fixed nodes, sources, receivers) are numpy arrays; nodal vectors that live on the GPU
(matvec operands, wavefields, traces) are torch CUDA float64 tensors, used only for
device memory and the stream.  If the library is missing this module raises on
import: there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libovfem.so")

OVFEM_FP64 = 0
OVFEM_INT8 = 1
OVFEM_INT8_BF16 = 2
OVFEM_FP64_SF = 3
PRECISIONS = {"fp64": OVFEM_FP64, "int8": OVFEM_INT8, "int8-bf16": OVFEM_INT8_BF16, "fp64-sf": OVFEM_FP64_SF}
ELEMENTS = {"ovfem": 0, "trilinear": 1}

# name -> (restype, argtypes); mirrors include/ovfem.h
_i32, _i64, _f64, _vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
SIGNATURES = {
    "ovfem_version": (_i32, []),
    "ovfem_last_error": (ctypes.c_char_p, []),
    "ovfem_create": (_i32, [ctypes.POINTER(_vp), _i64, _i64, _i64, _f64, _i32, _i32, _vp]),
    "ovfem_destroy": (_i32, [_vp]),
    "ovfem_set_precision": (_i32, [_vp, _i32]),
    "ovfem_set_model": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "ovfem_set_fixed_nodes": (_i32, [_vp, _vp]),
    "ovfem_set_dt": (_i32, [_vp, _f64]),
    "ovfem_set_sources": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i64]),
    "ovfem_set_receivers": (_i32, [_vp, _i32, _vp, _i64]),
    "ovfem_reset": (_i32, [_vp]),
    "ovfem_step": (_i32, [_vp, _i64]),
    "ovfem_matvec": (_i32, [_vp, _vp, _vp]),
    "ovfem_get_wavefield": (_i32, [_vp, _i32, _vp]),
    "ovfem_set_wavefield": (_i32, [_vp, _vp, _vp, _i64]),
    "ovfem_get_traces": (_i32, [_vp, _vp]),
    "ovfem_get_step": (_i32, [_vp, ctypes.POINTER(_i64)]),
    "ovfem_set_checkpointing": (_i32, [_vp, _i64, _i64]),
    "ovfem_adjoint": (_i32, [_vp, _vp, _vp, _vp]),
    "ovfem_set_element": (_i32, [_vp, _i32]),
    "ovfem_set_damping": (_i32, [_vp, _f64, _f64]),
    "ovfem_set_stages": (_i32, [_vp, _i32]),
    "ovfem_get_stages": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "ovfem_set_tuning": (_i32, [_vp, _i32, _i32, _i32]),
    "ovfem_get_tuning": (_i32, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "ovfem_autotune": (_i32, [_vp, _i32, ctypes.POINTER(_f64)]),
    "ovfem_set_tile_rows": (_i32, [_vp, _i32]),
    "ovfem_get_tile_rows": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "ovfem_batch_create": (_i32, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32]),
    "ovfem_batch_destroy": (_i32, [_vp]),
    "ovfem_batch_set_tuning": (_i32, [_vp, _i32]),
    "ovfem_batch_set_graph": (_i32, [_vp, _i32]),
    "ovfem_batch_step": (_i32, [_vp, _i64]),
    "ovfem_batch_step_noalloc": (_i32, [_vp, _i64]),
    "ovfem_check_finite": (_i32, [_vp, ctypes.POINTER(_i32)]),
    "ovfem_synchronize": (_i32, [_vp]),
}


class OvfemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libovfem status %d: %s" % (status, msg))
        self.status = status


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libovfem.so not built at %s (run __graft_entry__.build())" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = load_library()


def lib():
    return _LIB


def _check(status):
    if status != 0:
        raise OvfemError(status, _LIB.ovfem_last_error().decode())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _dev_f64(t, n, name, device):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("%s must be a contiguous CUDA float64 tensor" % name)
    if t.device.index != device:
        raise ValueError("%s is on cuda:%d, the solver on cuda:%d" % (name, t.device.index, device))
    if t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One OVFEM grid on the current GPU; all work on torch's current stream."""

    def __init__(self, nx, ny, nz, h, precision="fp64", n_shots=1, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.cuda.current_device()  # the library creates the solver there
        self.nx, self.ny, self.nz, self.h = int(nx), int(ny), int(nz), float(h)
        self.n_shots = int(n_shots)
        self.n_nodes = (self.nx + 1) * (self.ny + 1) * (self.nz + 1)
        self._h = ctypes.c_void_p()
        _check(_LIB.ovfem_create(ctypes.byref(self._h), self.nx, self.ny, self.nz, self.h, self.n_shots,
                                 PRECISIONS[precision], ctypes.c_void_p(stream.cuda_stream)))
        self.n_rec = 0
        self.rec_nt = 0
        self.dt = None
        # bumped by every call that changes the run the checkpoints and traces belong to
        # (model, problem, path, wavefield, stepping); the autograd wrapper compares it
        self.generation = 0

    def _touch(self):
        self.generation += 1

    def close(self):
        if self._h:
            _check(_LIB.ovfem_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --- configuration (host arrays)
    def set_precision(self, precision):
        self._touch()
        _check(_LIB.ovfem_set_precision(self._h, PRECISIONS[precision]))

    def set_model(self, lam, mu, rho, solid=None):
        la, lp = _host(lam, np.float64)
        ma, mp = _host(mu, np.float64)
        ra, rp = _host(rho, np.float64)
        n = self.nx * self.ny * self.nz
        for a in (la, ma, ra):
            if a.size != n:
                raise ValueError("material arrays must have nx*ny*nz entries")
        sp = None
        if solid is not None:
            sa, sp = _host(solid, np.uint8)
            if sa.size != n:
                raise ValueError("solid must have nx*ny*nz entries")
        self._touch()
        _check(_LIB.ovfem_set_model(self._h, lp, mp, rp, sp))

    def set_fixed_nodes(self, fixed):
        self._touch()
        if fixed is None:
            _check(_LIB.ovfem_set_fixed_nodes(self._h, None))
            return
        fa, fp = _host(fixed, np.uint8)
        if fa.size != self.n_nodes:
            raise ValueError("fixed must have one entry per node")
        _check(_LIB.ovfem_set_fixed_nodes(self._h, fp))

    def set_dt(self, dt):
        self._touch()
        _check(_LIB.ovfem_set_dt(self._h, float(dt)))
        self.dt = float(dt)

    def set_sources(self, node, comp, wavelet, shot=None):
        na, np_ = _host(node, np.int64)
        ca, cp = _host(comp, np.int32)
        wa, wp = _host(wavelet, np.float64)
        n = int(na.size)
        nt = int(wa.shape[-1]) if n else 0
        if n and wa.size != n * nt:
            raise ValueError("wavelet must be (n_sources, nt)")
        sp = None
        if shot is not None:
            sa, sp = _host(shot, np.int32)
        self._touch()
        _check(_LIB.ovfem_set_sources(self._h, n, np_, cp, sp, wp, nt))

    def set_receivers(self, node, nt_max):
        na, np_ = _host(node, np.int64)
        self._touch()
        _check(_LIB.ovfem_set_receivers(self._h, int(na.size), np_, int(nt_max)))
        self.n_rec, self.rec_nt = int(na.size), int(nt_max)

    @classmethod
    def from_workload(cls, wl, precision="fp64", receivers_nt=None, element="ovfem"):
        s = cls(wl.nx, wl.ny, wl.nz, wl.h, precision=precision, n_shots=wl.n_shots)
        if element != "ovfem":
            s.set_element(element)
        s.set_model(wl.lam, wl.mu, wl.rho, wl.solid)
        s.set_fixed_nodes(wl.fixed)
        s.set_dt(wl.dt)
        s.set_sources(wl.src_node, wl.src_comp, wl.wavelet, wl.src_shot)
        s.set_receivers(wl.rec_node, wl.nt if receivers_nt is None else receivers_nt)
        return s

    # --- stepping and data (device tensors)
    # The library runs everything on the solver's stream.  Device tensors the caller made
    # on another stream are ordered before the library's work on them, and the library's
    # outputs before the caller's stream goes on.
    def _order_in(self):
        import torch
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _order_out(self):
        import torch
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def reset(self):
        self._touch()
        _check(_LIB.ovfem_reset(self._h))

    def step(self, n=1):
        self._touch()
        _check(_LIB.ovfem_step(self._h, int(n)))

    def synchronize(self):
        _check(_LIB.ovfem_synchronize(self._h))

    def check_finite(self):
        """True if the current wavefield pair of every shot holds only finite values."""
        v = _i32()
        self._order_in()
        _check(_LIB.ovfem_check_finite(self._h, ctypes.byref(v)))
        return bool(v.value)

    def matvec(self, u, out=None):
        import torch
        n = 3 * self.n_nodes
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=self.device)
        self._order_in()
        _check(_LIB.ovfem_matvec(self._h, _dev_f64(u, n, "u", self.device), _dev_f64(out, n, "out", self.device)))
        self._order_out()
        return out

    def get_wavefield(self, which=0, out=None):
        """u^n (which=0) or u^{n-1} (which=1) of every shot, (n_shots * n_nodes * 3,)."""
        import torch
        n = self.n_shots * 3 * self.n_nodes
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=self.device)
        self._order_in()
        _check(_LIB.ovfem_get_wavefield(self._h, int(which), _dev_f64(out, n, "out", self.device)))
        self._order_out()
        return out

    def set_wavefield(self, un, unm1, step=0):
        n = self.n_shots * 3 * self.n_nodes
        self._order_in()
        self._touch()
        _check(_LIB.ovfem_set_wavefield(self._h, _dev_f64(un, n, "un", self.device),
                                        _dev_f64(unm1, n, "unm1", self.device), int(step)))

    def get_traces(self, out=None):
        import torch
        n = self.n_shots * self.n_rec * 3 * self.rec_nt
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float64, device=self.device)[:n]
        self._order_in()
        _check(_LIB.ovfem_get_traces(self._h, _dev_f64(out, n, "out", self.device) if n else None))
        self._order_out()
        return out.view(self.n_shots, self.n_rec, 3, self.rec_nt)

    def set_checkpointing(self, every, max_steps):
        self._touch()
        _check(_LIB.ovfem_set_checkpointing(self._h, int(every), int(max_steps)))

    def adjoint(self, residual):
        """(g_lam, g_mu) as CUDA float64 tensors (nz, ny, nx) for dJ/d(traces) = residual
        ([shot][receiver][3][nt], the traces' layout); with several shots, the gradient of
        a misfit summed over them."""
        import torch
        n = self.n_shots * self.n_rec * 3 * self.rec_nt
        r = residual.reshape(-1)
        ne = self.nx * self.ny * self.nz
        g_lam = torch.empty(ne, dtype=torch.float64, device=self.device)
        g_mu = torch.empty(ne, dtype=torch.float64, device=self.device)
        self._order_in()
        _check(_LIB.ovfem_adjoint(self._h, _dev_f64(r, n, "residual", self.device),
                                  _dev_f64(g_lam, ne, "g_lam", self.device), _dev_f64(g_mu, ne, "g_mu", self.device)))
        self._order_out()
        shape = (self.nz, self.ny, self.nx)
        return g_lam.view(shape), g_mu.view(shape)

    def get_step(self):
        v = ctypes.c_int64()
        _check(_LIB.ovfem_get_step(self._h, ctypes.byref(v)))
        return v.value

    # --- element type (before the model)
    def set_element(self, element):
        self._touch()
        _check(_LIB.ovfem_set_element(self._h, ELEMENTS[element]))

    # --- Rayleigh damping C = alpha M + beta K
    def set_damping(self, alpha, beta):
        self._touch()
        _check(_LIB.ovfem_set_damping(self._h, float(alpha), float(beta)))

    # --- digit stages of the INT8 form
    def set_stages(self, stages):
        self._touch()
        _check(_LIB.ovfem_set_stages(self._h, int(stages)))

    def get_stages(self):
        v = _i32()
        _check(_LIB.ovfem_get_stages(self._h, ctypes.byref(v)))
        return v.value

    # --- launch configuration
    def set_tuning(self, chunk_planes=16, persistent_groups=0, graph_steps=0, tile_rows=None):
        self._touch()
        if tile_rows is not None:
            _check(_LIB.ovfem_set_tile_rows(self._h, int(tile_rows)))
        _check(_LIB.ovfem_set_tuning(self._h, int(chunk_planes), int(persistent_groups), int(graph_steps)))

    def get_tuning(self):
        a, b, c, r = _i32(), _i32(), _i32(), _i32()
        _check(_LIB.ovfem_get_tuning(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        _check(_LIB.ovfem_get_tile_rows(self._h, ctypes.byref(r)))
        return {"chunk_planes": a.value, "persistent_groups": b.value, "graph_steps": c.value, "tile_rows": r.value}

    def autotune(self, steps=20):
        """Pick the fastest launch configuration; returns its ms per step."""
        ms = _f64()
        self._touch()
        _check(_LIB.ovfem_autotune(self._h, int(steps), ctypes.byref(ms)))
        return ms.value


class Batch:
    """Solvers of uneven sizes stepped together, one kernel launch per step."""

    def __init__(self, solvers):
        self.members = list(solvers)
        arr = (_vp * len(self.members))(*[m._h.value for m in self.members])
        self._h = ctypes.c_void_p()
        _check(_LIB.ovfem_batch_create(ctypes.byref(self._h), arr, len(self.members)))

    def set_tuning(self, persistent_groups=0):
        _check(_LIB.ovfem_batch_set_tuning(self._h, int(persistent_groups)))

    def set_graph(self, graph_steps):
        """Replay blocks of graph_steps (a multiple of 6) steps from a captured graph."""
        _check(_LIB.ovfem_batch_set_graph(self._h, int(graph_steps)))

    def step(self, n=1):
        for m in self.members:
            m._touch()
        _check(_LIB.ovfem_batch_step(self._h, int(n)))

    def step_noalloc(self, n=1):
        """step() with the argument tables in the library's fixed device array (no device
        allocation); every member must have stepped since it was last changed."""
        for m in self.members:
            m._touch()
        _check(_LIB.ovfem_batch_step_noalloc(self._h, int(n)))

    def close(self):
        if self._h:
            _check(_LIB.ovfem_batch_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
