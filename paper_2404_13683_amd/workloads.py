"""Seeded synthetic inputs for the voxel elastic-wave stepper.

Shared by the tests, the benchmark and the smoke check, and consumed identically by
the HIP library and the CPU oracle.  This module holds none of the method's
arithmetic (no element matrices, no mass, no stepping): only grid sizes, material
fields, boundary flags, source time functions and receiver positions.

Conventions: elements are (nz, ny, nx) arrays, nodes (nz+1, ny+1, nx+1); the flat
node id is i + (nx+1) (j + (ny+1) k); z points up and k = nz is the top surface.
Unless a recipe says otherwise Vp = 2 Vs, so lam = 2 rho Vs^2 and mu = rho Vs^2,
the source is a z-directed Ricker wavelet with t0 = 1.2 / f0 and unit amplitude,
and dt = 0.5 h / max Vp.  Every face except the top is fixed (all three DOFs).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    h: float
    lam: np.ndarray            # (nz, ny, nx) float64, per element
    mu: np.ndarray             # (nz, ny, nx) float64
    rho: np.ndarray            # (nz, ny, nx) float64
    fixed: np.ndarray          # (nz+1, ny+1, nx+1) uint8, 1 = all three DOFs held at zero
    dt: float
    nt: int
    src_node: np.ndarray       # (n_src,) int64 flat node ids
    src_comp: np.ndarray       # (n_src,) int32 component 0/1/2
    src_shot: np.ndarray       # (n_src,) int32 shot index
    wavelet: np.ndarray        # (n_src, nt) float64 force at step n (time n dt)
    rec_node: np.ndarray       # (n_rec,) int64 flat node ids (same receivers for every shot)
    n_shots: int = 1
    solid: Optional[np.ndarray] = None   # (nz, ny, nx) uint8, None = all solid
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self):
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def n_elements(self):
        return self.nx * self.ny * self.nz

    def touched_nodes(self):
        """Nodes touching at least one solid element (geometric, no physics)."""
        nz, ny, nx = self.nz, self.ny, self.nx
        s = np.ones((nz, ny, nx), bool) if self.solid is None else self.solid.astype(bool)
        t = np.zeros((nz + 1, ny + 1, nx + 1), bool)
        for dk in (0, 1):
            for dj in (0, 1):
                for di in (0, 1):
                    t[dk:dk + nz, dj:dj + ny, di:di + nx] |= s
        return t

    def free_dof(self):
        """3 x (nodes that are not fixed and touch solid): the DOFs updated each step."""
        return int(3 * np.count_nonzero(self.touched_nodes() & (self.fixed == 0)))


def node_id(i, j, k, nx, ny):
    return int(i) + (nx + 1) * (int(j) + (ny + 1) * int(k))


def ricker(nt, dt, f0, t0=None, amp=1.0):
    """Ricker wavelet (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2) at t = n dt."""
    t0 = 1.2 / f0 if t0 is None else t0
    t = np.arange(nt) * dt - t0
    a = (np.pi * f0 * t) ** 2
    return amp * (1.0 - 2.0 * a) * np.exp(-a)


def box_fixed(nx, ny, nz):
    """Fixed flags: all faces except the top (k = nz)."""
    f = np.zeros((nz + 1, ny + 1, nx + 1), np.uint8)
    f[0] = 1
    f[:, 0, :] = 1
    f[:, ny, :] = 1
    f[:, :, 0] = 1
    f[:, :, nx] = 1
    return f


def lame_from_velocities(vp, vs, rho):
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return lam, mu


def stable_dt(h, lam, mu, rho, cfl=0.5):
    vp = np.sqrt((lam + 2.0 * mu) / rho)
    return float(cfl * h / vp.max())


def surface_nodes(rng, n, nx, ny, nz, margin=1, exclude=()):
    """n distinct seeded top-surface nodes away from the fixed side faces."""
    out = []
    taken = set(int(e) for e in exclude)
    while len(out) < n:
        i = int(rng.integers(margin, nx - margin + 1))
        j = int(rng.integers(margin, ny - margin + 1))
        nd = node_id(i, j, nz, nx, ny)
        if nd not in taken:
            taken.add(nd)
            out.append(nd)
    return np.array(out, dtype=np.int64)


def smooth_perturbation(rng, shape, sigma_vox, amp):
    """Seeded white noise convolved with a Gaussian (sigma in voxels), scaled to max |d| = amp."""
    from scipy.ndimage import gaussian_filter
    w = rng.standard_normal(shape)
    s = gaussian_filter(w, sigma=sigma_vox, mode="reflect", truncate=3.0)
    return amp * s / np.abs(s).max()


def homogeneous_c1(nx=16, ny=16, nz=16, h=1.0, rho=2000.0, vp=2000.0, vs=1000.0,
                   f0=50.0, nt=200, n_rec=8, seed=1):
    """Homogeneous cube, centre z-force, free top, other faces fixed, dt at 0.5 CFL.

    Default: 16^3 voxels, h = 1 m, rho = 2000 kg/m^3, Vp = 2000 m/s, Vs = 1000 m/s,
    Ricker f0 = 50 Hz at the centre node, 200 steps, 8 seeded top-surface receivers.
    """
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    lam0, mu0 = lame_from_velocities(vp, vs, rho)
    lam = np.full(shape, lam0)
    mu = np.full(shape, mu0)
    rr = np.full(shape, rho)
    dt = stable_dt(h, lam, mu, rr)
    src = np.array([node_id(nx // 2, ny // 2, nz // 2, nx, ny)], np.int64)
    return Workload("c1-homogeneous", nx, ny, nz, h, lam, mu, rr, box_fixed(nx, ny, nz), dt, nt,
                    src, np.array([2], np.int32), np.array([0], np.int32),
                    ricker(nt, dt, f0)[None, :],
                    surface_nodes(rng, n_rec, nx, ny, nz), meta=dict(f0=f0, seed=seed))


def layered_medium(rng, nx, ny, nz, h, vs_layers=(300.0, 800.0, 2000.0),
                   rho_layers=(1800.0, 2100.0, 2500.0), fractions=(0.25, 0.25, 0.5),
                   pert=0.10, corr_len=50.0):
    """Three horizontal layers (top to bottom) with smooth seeded lam/mu perturbations."""
    shape = (nz, ny, nx)
    vs = np.empty(shape)
    rho = np.empty(shape)
    # thickness in voxels, from the top
    t1 = int(round(fractions[0] * nz))
    t2 = int(round(fractions[1] * nz))
    bounds = [nz, nz - t1, nz - t1 - t2, 0]
    for layer in range(3):
        lo, hi = bounds[layer + 1], bounds[layer]
        vs[lo:hi] = vs_layers[layer]
        rho[lo:hi] = rho_layers[layer]
    lam, mu = lame_from_velocities(2.0 * vs, vs, rho)
    if pert > 0:
        sig = corr_len / h
        lam = lam * (1.0 + smooth_perturbation(rng, shape, sig, pert))
        mu = mu * (1.0 + smooth_perturbation(rng, shape, sig, pert))
    return lam, mu, rho


def layered_c2(nx=256, ny=256, nz=128, h=5.0, f0=5.0, nt=2000, n_rec=8, seed=2, pert=0.10):
    """Single shot on three horizontal layers with smooth +-10 % lam/mu perturbation.

    Default 256 x 256 x 128 voxels (8.4 M elements), h = 5 m, layers 32/32/64 voxels
    from the top with Vs 300/800/2000 m/s, Vp = 2 Vs, rho 1800/2100/2500 kg/m^3,
    Gaussian-correlated (L = 50 m) perturbation, Ricker f0 = 5 Hz at the top-surface
    centre, 2000 steps, 8 seeded top-surface receivers.
    """
    rng = np.random.default_rng(seed)
    lam, mu, rho = layered_medium(rng, nx, ny, nz, h, pert=pert)
    dt = stable_dt(h, lam, mu, rho)
    src = np.array([node_id(nx // 2, ny // 2, nz, nx, ny)], np.int64)
    return Workload("c2-layered", nx, ny, nz, h, lam, mu, rho, box_fixed(nx, ny, nz), dt, nt,
                    src, np.array([2], np.int32), np.array([0], np.int32),
                    ricker(nt, dt, f0)[None, :],
                    surface_nodes(rng, n_rec, nx, ny, nz, exclude=src),
                    meta=dict(f0=f0, seed=seed))


def shots_c3(nx=128, ny=128, nz=64, h=5.0, n_shots=64, f0=5.0, nt=1000, n_rec=8, seed=3):
    """Many independent shots on the layered medium scaled to 128 x 128 x 64 voxels.

    Each shot has one z-directed Ricker source at a seeded top-surface node; all shots
    share the same 8 receivers.
    """
    rng = np.random.default_rng(seed)
    lam, mu, rho = layered_medium(rng, nx, ny, nz, h)
    dt = stable_dt(h, lam, mu, rho)
    src = surface_nodes(rng, n_shots, nx, ny, nz, margin=2)
    w = np.tile(ricker(nt, dt, f0)[None, :], (n_shots, 1))
    return Workload("c3-shots", nx, ny, nz, h, lam, mu, rho, box_fixed(nx, ny, nz), dt, nt,
                    src, np.full(n_shots, 2, np.int32), np.arange(n_shots, dtype=np.int32), w,
                    surface_nodes(rng, n_rec, nx, ny, nz, exclude=src), n_shots=n_shots,
                    meta=dict(f0=f0, seed=seed))


def uneven_domains_c3(n_domains=16, smallest=(32, 32, 32), largest=(160, 160, 80), h=5.0,
                      f0=5.0, nt=1000, n_rec=8, seed=4):
    """A batch of layered domains of seeded uneven sizes (first smallest, last largest)."""
    rng = np.random.default_rng(seed)
    sizes = [tuple(smallest)]
    for _ in range(n_domains - 2):
        sizes.append((int(rng.integers(smallest[0], largest[0] + 1)),
                      int(rng.integers(smallest[1], largest[1] + 1)),
                      int(rng.integers(smallest[2], largest[2] + 1))))
    sizes.append(tuple(largest))
    out = []
    for d, (nx, ny, nz) in enumerate(sizes[:n_domains]):
        wl = layered_c2(nx, ny, nz, h=h, f0=f0, nt=nt, n_rec=n_rec, seed=1000 * seed + d)
        wl.name = "c3-domain-%d" % d
        out.append(wl)
    return out


def adjoint_c4(nx=96, ny=96, nz=96, h=5.0, f0=5.0, nt=1000, n_rec=32, seed=5, pert=0.15,
               vs=800.0, vp=1600.0, rho=2100.0):
    """Adjoint workload: returns (true model, homogeneous start model) sharing geometry.

    Start model homogeneous (Vs 800, Vp 1600, rho 2100); true model = start x (1 + d)
    for independent smooth lam/mu perturbations with max |d| = 0.15, L = 50 m.
    Centre-surface z-source, 32 seeded surface receivers, dt from the true model.
    """
    rng = np.random.default_rng(seed)
    shape = (nz, ny, nx)
    lam0, mu0 = lame_from_velocities(vp, vs, rho)
    lam_s = np.full(shape, lam0)
    mu_s = np.full(shape, mu0)
    rr = np.full(shape, rho)
    sig = 50.0 / h
    lam_t = lam_s * (1.0 + smooth_perturbation(rng, shape, sig, pert))
    mu_t = mu_s * (1.0 + smooth_perturbation(rng, shape, sig, pert))
    dt = stable_dt(h, lam_t, mu_t, rr)
    src = np.array([node_id(nx // 2, ny // 2, nz, nx, ny)], np.int64)
    rec = surface_nodes(rng, n_rec, nx, ny, nz, exclude=src)
    common = dict(nx=nx, ny=ny, nz=nz, h=h, rho=rr, fixed=box_fixed(nx, ny, nz), dt=dt, nt=nt,
                  src_node=src, src_comp=np.array([2], np.int32), src_shot=np.array([0], np.int32),
                  wavelet=ricker(nt, dt, f0)[None, :], rec_node=rec, meta=dict(f0=f0, seed=seed))
    true = Workload("c4-true", lam=lam_t, mu=mu_t, **common)
    start = Workload("c4-start", lam=lam_s, mu=mu_s, **common)
    return true, start


def fractal_surface(rng, nx, ny, hurst=0.7, relief=40.0):
    """Seeded fractal height field (nx x ny cell centres), max |height - mean| = relief.

    Spectral synthesis: random phases with amplitude |k|^-(hurst + 1), i.e. the power
    spectrum |k|^-(2 hurst + 2) of a fractional Brownian surface.
    """
    kx = np.fft.fftfreq(nx)[None, :]
    ky = np.fft.fftfreq(ny)[:, None]
    k = np.sqrt(kx * kx + ky * ky)
    k[0, 0] = np.inf
    amp = k ** -(hurst + 1.0)
    spec = amp * np.exp(2j * np.pi * rng.random((ny, nx)))
    z = np.real(np.fft.ifft2(spec))
    z -= z.mean()
    return relief * z / np.abs(z).max()


def top_solid_nodes(rng, n, solid, margin=1, exclude=()):
    """n distinct seeded nodes on the top of the solid: node (i, j, kt + 1) above the
    highest solid voxel kt of column (i, j)."""
    nz, ny, nx = solid.shape
    out = []
    taken = set(int(e) for e in exclude)
    while len(out) < n:
        i = int(rng.integers(margin, nx - margin))
        j = int(rng.integers(margin, ny - margin))
        col = np.nonzero(solid[:, j, i])[0]
        if col.size == 0:
            continue
        nd = node_id(i, j, col.max() + 1, nx, ny)
        if nd not in taken:
            taken.add(nd)
            out.append(nd)
    return np.array(out, dtype=np.int64)


def topography_c5(nx=512, ny=512, nz=256, h=2.0, f0=5.0, nt=4000, n_rec=8, seed=6, relief=None,
                  hurst=0.7, vs=(200.0, 600.0, 1500.0), rho=(1800.0, 2100.0, 2500.0)):
    """Fractal free-surface topography over a nested two-bowl basin in bedrock.

    Default 512 x 512 x 256 voxels, h = 2 m.  Surface: seeded fractal height field
    (Hurst 0.7) of relief +-40 m (scaled with nz for smaller grids) around a mean
    elevation 1.25 relief below the top of the box; a voxel is solid if its centre lies
    below the surface (air voxels removed).  Materials (Vp = 2 Vs): bedrock Vs 1500,
    rho 2500; a seeded ellipsoidal bowl under the mean surface with Vs 600, rho 2100;
    inside it a shallower nested bowl with Vs 200, rho 1800.  Air voxels carry bedrock
    values (unused).  Centre-surface z-force, Ricker f0, 8 seeded receivers on the
    surface, dt = 0.5 h / max Vp.
    """
    rng = np.random.default_rng(seed)
    if relief is None:
        relief = 40.0 * nz / 256.0
    top = nz * h
    mean_surface = top - 1.25 * relief
    surf = mean_surface + fractal_surface(rng, nx, ny, hurst, relief)      # (ny, nx)
    zc = (np.arange(nz) + 0.5) * h
    yc = (np.arange(ny) + 0.5) * h
    xc = (np.arange(nx) + 0.5) * h
    solid = (zc[:, None, None] < surf[None, :, :]).astype(np.uint8)
    Lx, Ly = nx * h, ny * h
    cx, cy = rng.uniform(0.35, 0.65) * Lx, rng.uniform(0.35, 0.65) * Ly
    ax, ay = rng.uniform(0.2, 0.35) * Lx, rng.uniform(0.2, 0.35) * Ly
    az = rng.uniform(0.25, 0.4) * mean_surface
    dx = ((xc - cx) / ax)[None, None, :]
    dy = ((yc - cy) / ay)[None, :, None]
    dz = ((mean_surface - zc) / az)[:, None, None]
    r_outer = dx * dx + dy * dy + dz * dz
    r_inner = (dx / 0.6) ** 2 + (dy / 0.6) ** 2 + (dz / 0.4) ** 2
    vs_f = np.full((nz, ny, nx), vs[2])
    rho_f = np.full((nz, ny, nx), rho[2])
    outer = (r_outer < 1.0) & (zc[:, None, None] < mean_surface + relief + h)
    vs_f[outer] = vs[1]
    rho_f[outer] = rho[1]
    inner = outer & (r_inner < 1.0)
    vs_f[inner] = vs[0]
    rho_f[inner] = rho[0]
    del r_outer, r_inner, outer, inner
    lam, mu = lame_from_velocities(2.0 * vs_f, vs_f, rho_f)
    del vs_f
    dt = float(0.5 * h / (2.0 * max(vs)))
    col = np.nonzero(solid[:, ny // 2, nx // 2])[0]
    src = np.array([node_id(nx // 2, ny // 2, col.max() + 1, nx, ny)], np.int64)
    rec = top_solid_nodes(rng, n_rec, solid, exclude=src)
    return Workload("c5-topography", nx, ny, nz, h, lam, mu, rho_f, box_fixed(nx, ny, nz), dt, nt,
                    src, np.array([2], np.int32), np.array([0], np.int32),
                    ricker(nt, dt, f0)[None, :], rec, solid=solid,
                    meta=dict(f0=f0, seed=seed, relief=relief, hurst=hurst))


def single_shot(w, shot):
    """The one-shot workload made of shot `shot` of a multi-shot workload."""
    import dataclasses
    sel = np.nonzero(np.asarray(w.src_shot) == shot)[0]
    return dataclasses.replace(w, name="%s-shot%d" % (w.name, shot), src_node=w.src_node[sel],
                               src_comp=w.src_comp[sel], src_shot=np.zeros(len(sel), np.int32),
                               wavelet=w.wavelet[sel], n_shots=1)


def with_surface_shots(w, n, seed=0):
    """w with n shots: shot 0 is w's one-shot source set, shots 1 .. n-1 the same first
    source (component, wavelet) moved to seeded top-surface nodes away from the receivers."""
    import dataclasses
    if w.n_shots != 1 or n < 1:
        raise ValueError("with_surface_shots: needs a one-shot workload and n >= 1")
    rng = np.random.default_rng(seed)
    extra = surface_nodes(rng, n - 1, w.nx, w.ny, w.nz, exclude=np.concatenate([w.src_node, w.rec_node]))
    return dataclasses.replace(
        w, name="%s-%dshots" % (w.name, n), n_shots=n,
        src_node=np.concatenate([w.src_node, extra]),
        src_comp=np.concatenate([w.src_comp, np.full(n - 1, w.src_comp[0], np.int32)]),
        src_shot=np.concatenate([np.asarray(w.src_shot, np.int32), np.arange(1, n, dtype=np.int32)]),
        wavelet=np.concatenate([w.wavelet, np.repeat(w.wavelet[:1], n - 1, axis=0)]))


def random_field(shape, seed, scale=1.0):
    """Seeded standard-normal nodal field (for per-matvec parity)."""
    return scale * np.random.default_rng(seed).standard_normal(shape)
