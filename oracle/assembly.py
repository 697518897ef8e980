"""Structured-grid OVFEM operator, stepper and adjoint (oracle; test infrastructure only).

Grid conventions (shared with the inputs, not with any implementation):
  * elements (nz, ny, nx), element (i, j, k) spans nodes i..i+1, j..j+1, k..k+1;
  * nodal arrays (nz+1, ny+1, nx+1, 3); flat node id = i + (nx+1) (j + (ny+1) k);
  * local corner alpha = di + 2 dj + 4 dk, element DOF 3 alpha + c (see element.py).

What is computed, all in float64:
  * f = K u = sum_e  scatter_e( K_e u_e ),  K_e = h (lam_e K_lam + mu_e K_mu)
    (Sec. 2, Eq. (2) assembled from the Eq. (5) element matrices);
  * nodal mass m = sum_e rho_e (phi phi)_e, i.e. rho_e h^3 / 8 from each touching
    solid element (Sec. 2, Eq. (6): diagonal without approximation);
  * central-difference stepping (Sec. 2, Eq. (3), solved for u^{it+1} as in
    Sec. 3, Eq. (19) with the force sign of Eq. (3)):
        u^{n+1} = 2 u^n - u^{n-1} + dt^2 m^{-1} (F^n - K u^n)   on free DOFs,
    fixed DOFs (and nodes with no mass) held at zero;
  * optional Rayleigh damping C = alpha M + beta K (the paper's experiment uses it,
    Sec. 3; its time discretization is not printed).  Reading: the mass-proportional
    velocity is centred and the stiffness-proportional one taken backward, which keeps
    the step explicit with one K product:
        M (u^{n+1} - 2u^n + u^{n-1}) / dt^2 + alpha M (u^{n+1} - u^{n-1}) / (2 dt)
          + beta K (u^n - u^{n-1}) / dt + K u^n = F^n,
    i.e. (1 + alpha dt/2) u^{n+1} = 2u^n - (1 - alpha dt/2) u^{n-1}
          + dt^2 m^{-1} (F^n - K (u^n + (beta/dt) (u^n - u^{n-1})));
  * receivers record u^{n+1} after step n;
  * discrete energy, discrete adjoint of a trace misfit, and the error measure of
    Sec. 3, Eq. (18).
"""
import numpy as np

from .element import ovfem_reference, trilinear_reference


def corner_slices(nx, ny, nz):
    """For corner alpha = di + 2 dj + 4 dk: the node-array slice holding that corner of every element."""
    out = []
    for alpha in range(8):
        di, dj, dk = alpha & 1, (alpha >> 1) & 1, (alpha >> 2) & 1
        out.append((slice(dk, dk + nz), slice(dj, dj + ny), slice(di, di + nx)))
    return out


def gather(u, nx, ny, nz):
    """Element displacement vectors u_e: (nz, ny, nx, 24), DOF 3 alpha + c."""
    sl = corner_slices(nx, ny, nz)
    return np.concatenate([u[s] for s in sl], axis=-1)


def scatter_add(f, ye, nx, ny, nz):
    """f[node] += sum over elements of their local vectors ye (nz, ny, nx, 24)."""
    for alpha, s in enumerate(corner_slices(nx, ny, nz)):
        f[s] += ye[..., 3 * alpha:3 * alpha + 3]
    return f


def element_matvec(ue, lam, mu, h, K=None):
    """K_e u_e = h (lam_e K_lam u_e + mu_e K_mu u_e) for every element."""
    Kl, Km = ovfem_reference() if K is None else K
    return h * (lam[..., None] * (ue @ Kl.T) + mu[..., None] * (ue @ Km.T))


def matvec(u, lam, mu, h, K=None):
    """Assembled K u on the whole node array (no boundary conditions applied).

    Elements with lam = mu = 0 (e.g. removed voxels) contribute nothing.
    """
    nz, ny, nx = lam.shape
    f = np.zeros_like(u)
    ye = element_matvec(gather(u, nx, ny, nz), lam, mu, h, K)
    return scatter_add(f, ye, nx, ny, nz)


def nodal_mass(rho, h, solid=None):
    """Diagonal mass per node: sum over touching solid elements of rho_e h^3 / 8."""
    nz, ny, nx = rho.shape
    r = rho if solid is None else np.where(solid, rho, 0.0)
    m = np.zeros((nz + 1, ny + 1, nx + 1))
    for s in corner_slices(nx, ny, nz):
        m[s] += r * (h ** 3 / 8.0)
    return m


def free_mask(fixed, mass):
    """Nodes that move: not fixed and with positive mass."""
    return (fixed == 0) & (mass > 0)


def forcing(shape, src_node, src_comp, amp):
    """Nodal force array with amp[s] applied at (src_node[s], src_comp[s])."""
    F = np.zeros(shape)
    flat = F.reshape(-1, 3)
    for nd, c, a in zip(src_node, src_comp, amp):
        flat[int(nd), int(c)] += a
    return F


def rayleigh_coefficients(zeta, f1, f2):
    """(alpha, beta) of Rayleigh damping C = alpha M + beta K with damping ratio zeta at
    the frequencies f1 and f2: a mode of angular frequency w is damped with ratio
    alpha / (2 w) + beta w / 2, which equals zeta at w1 = 2 pi f1 and w2 = 2 pi f2."""
    w1, w2 = 2.0 * np.pi * f1, 2.0 * np.pi * f2
    return 2.0 * zeta * w1 * w2 / (w1 + w2), 2.0 * zeta / (w1 + w2)


class Model:
    """Inputs of one simulation, plus the oracle's own derived mass."""

    def __init__(self, lam, mu, rho, h, fixed, dt, solid=None, alpha=0.0, beta=0.0, element="ovfem"):
        self.lam = np.asarray(lam, dtype=np.float64)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.rho = np.asarray(rho, dtype=np.float64)
        self.solid = None if solid is None else np.asarray(solid).astype(bool)
        if self.solid is not None:
            self.lam = np.where(self.solid, self.lam, 0.0)
            self.mu = np.where(self.solid, self.mu, 0.0)
        self.h = float(h)
        self.dt = float(dt)
        self.nz, self.ny, self.nx = self.lam.shape
        self.mass = nodal_mass(self.rho, self.h, self.solid)
        self.free = free_mask(np.asarray(fixed), self.mass)
        self.node_shape = (self.nz + 1, self.ny + 1, self.nx + 1, 3)
        # dt^2 / m on free nodes, 0 elsewhere
        self.a = np.zeros(self.node_shape[:3])
        self.a[self.free] = self.dt ** 2 / self.mass[self.free]
        self.alpha = float(alpha)
        self.beta = float(beta)
        # element matrices: OVFEM (Eq. (5)) or the lumped trilinear element ("VFEM"),
        # both with the same diagonal mass rho h^3 / 8 per node and element
        self.Kref = ovfem_reference() if element == "ovfem" else trilinear_reference()

    def K(self, u):
        return matvec(u, self.lam, self.mu, self.h, self.Kref)

    def step(self, u, u_prev, F):
        """One central-difference step; returns u^{n+1}."""
        if self.alpha == 0.0 and self.beta == 0.0:
            un = 2.0 * u - u_prev + self.a[..., None] * (F - self.K(u))
        else:
            ad = 0.5 * self.alpha * self.dt
            w = u + (self.beta / self.dt) * (u - u_prev)
            un = (2.0 * u - (1.0 - ad) * u_prev + self.a[..., None] * (F - self.K(w))) / (1.0 + ad)
        un[~self.free] = 0.0
        return un


def simulate(model, nt, src_node, src_comp, wavelet, rec_node, u0=None, u_prev=None,
             keep_states=False):
    """Run nt steps from (u^0, u^{-1}) (zero by default).

    wavelet[s, n] is the force of source s at step n (time n dt).
    Returns (traces (n_rec, 3, nt), u^nt, u^{nt-1}, states or None) where traces[r, c, n]
    is u^{n+1} at receiver r, component c, and states[n] = u^n for n = 0..nt.
    """
    u = np.zeros(model.node_shape) if u0 is None else np.array(u0, dtype=np.float64)
    up = np.zeros(model.node_shape) if u_prev is None else np.array(u_prev, dtype=np.float64)
    rec = np.asarray(rec_node, dtype=np.int64)
    traces = np.zeros((len(rec), 3, nt))
    states = [u.copy()] if keep_states else None
    for n in range(nt):
        F = forcing(model.node_shape, src_node, src_comp, wavelet[:, n])
        un = model.step(u, up, F)
        up, u = u, un
        traces[:, :, n] = u.reshape(-1, 3)[rec]
        if keep_states:
            states.append(u.copy())
    return traces, u, up, states


def energy(model, u_next, u):
    """Discrete energy E^{n+1/2} = 1/2 v^T M v + 1/2 (u^{n+1})^T K u^n, v = (u^{n+1} - u^n) / dt.

    Conserved by the unforced central-difference scheme because M is diagonal and
    K symmetric (Sec. 2, Eq. (3)); fixed DOFs are zero so the sums run over free DOFs.
    """
    v = (u_next - u) / model.dt
    kin = 0.5 * np.sum(model.mass[..., None] * model.free[..., None] * v * v)
    pot = 0.5 * np.sum(u_next * model.K(u))
    return kin + pot


def element_forms(ue, we, h, K=None):
    """Per element: h w_e^T K_lam u_e and h w_e^T K_mu u_e (the d(w^T K u)/d lam_e, mu_e)."""
    Kl, Km = ovfem_reference() if K is None else K
    return (h * np.einsum("...i,...i->...", we, ue @ Kl.T),
            h * np.einsum("...i,...i->...", we, ue @ Km.T))


def misfit(traces, d_obs):
    """J = 1/2 sum over receivers, components and steps of (u_sim - d_obs)^2."""
    r = traces - d_obs
    return 0.5 * float(np.sum(r * r))


def adjoint_gradient(model, nt, src_node, src_comp, wavelet, rec_node, d_obs, ckpt_every=None):
    """Gradient of J = misfit(traces, d_obs) with respect to per-element lam and mu.

    Discrete adjoint of the stepper (derived from the Lagrangian of the recursion
    u^{n+1} = (2I - A K) u^n - u^{n-1} + A F^n with A = dt^2 M^{-1} on free DOFs):
        w^{N+1} = w^{N+2} = 0,
        w^m = 2 w^{m+1} - w^{m+2} - A K w^{m+1} + A R^T r^{m-1},   m = N .. 1,
    with r^{n} = traces at step n minus d_obs, and
        dJ/dlam_e = - sum_{m=1}^{N} h (w_e^m)^T K_lam u_e^{m-1}   (same with K_mu).
    With Rayleigh damping the recursion is u^{n+1} = P u^n + Q u^{n-1} + Ah F^n with
    P = c1 I - (1+b) Ah K, Q = -c2 I + b Ah K (c1 = 2/(1+a), c2 = (1-a)/(1+a),
    a = alpha dt/2, b = beta/dt, Ah = A/(1+a)); the same Lagrangian argument with
    w = Ah lambda gives
        w^m = c1 w^{m+1} - c2 w^{m+2} - Ah K ((1+b) w^{m+1} - b w^{m+2}) + Ah R^T r^{m-1},
        dJ/dlam_e = - sum_m h (w_e^m)^T K_lam ((1+b) u^{m-1} - b u^{m-2})_e.
    Forward states are kept every ckpt_every steps and recomputed per segment
    (ckpt_every=None keeps all of them).
    Returns (J, g_lam, g_mu).
    """
    damped = model.alpha != 0.0 or model.beta != 0.0
    ad = 0.5 * model.alpha * model.dt
    bd = model.beta / model.dt
    rec = np.asarray(rec_node, dtype=np.int64)
    nx, ny, nz = model.nx, model.ny, model.nz
    every = nt if ckpt_every is None else int(ckpt_every)
    # forward pass: traces and checkpoints (u^s, u^{s-1}) at s = 0, every, 2 every, ...
    u = np.zeros(model.node_shape)
    up = np.zeros(model.node_shape)
    ckpts = {}
    traces = np.zeros((len(rec), 3, nt))
    for n in range(nt):
        if n % every == 0:
            ckpts[n] = (u.copy(), up.copy())
        F = forcing(model.node_shape, src_node, src_comp, wavelet[:, n])
        un = model.step(u, up, F)
        up, u = u, un
        traces[:, :, n] = u.reshape(-1, 3)[rec]
    J = misfit(traces, d_obs)
    resid = traces - d_obs
    A = model.a[..., None]

    g_lam = np.zeros(model.lam.shape)
    g_mu = np.zeros(model.mu.shape)
    w1 = np.zeros(model.node_shape)  # w^{m+1}
    w2 = np.zeros(model.node_shape)  # w^{m+2}
    seg_starts = sorted(ckpts.keys(), reverse=True)
    for s in seg_starts:
        e = min(s + every, nt)
        # recompute u^s .. u^e from the checkpoint (states[0] = u^{s-1} when damped)
        u, up = ckpts[s]
        states = ([up.copy()] if damped else []) + [u.copy()]
        o = 1 if damped else 0
        for n in range(s, e):
            F = forcing(model.node_shape, src_node, src_comp, wavelet[:, n])
            un = model.step(u, up, F)
            up, u = u, un
            states.append(u.copy())
        # adjoint steps m = e .. s+1 use u^{m-1} = states[m-1-s+o]
        for m in range(e, s, -1):
            src = np.zeros(model.node_shape)
            flat = src.reshape(-1, 3)
            np.add.at(flat, rec, resid[:, :, m - 1])
            if damped:
                Ah = A / (1.0 + ad)
                wm = (2.0 * w1 - (1.0 - ad) * w2) / (1.0 + ad) - Ah * model.K((1.0 + bd) * w1 - bd * w2) + Ah * src
                uh = (1.0 + bd) * states[m - 1 - s + o] - bd * states[m - 2 - s + o]
            else:
                wm = 2.0 * w1 - w2 - A * model.K(w1) + A * src
                uh = states[m - 1 - s]
            wm[~model.free] = 0.0
            gl, gm = element_forms(gather(uh, nx, ny, nz),
                                   gather(wm, nx, ny, nz), model.h, model.Kref)
            g_lam -= gl
            g_mu -= gm
            w2, w1 = w1, wm
    if model.solid is not None:
        g_lam = np.where(model.solid, g_lam, 0.0)
        g_mu = np.where(model.solid, g_mu, 0.0)
    return J, g_lam, g_mu


def err_measure(obs, ref):
    """Error of Sec. 3, Eq. (18): mean over channels of sum_t (obs - ref)^2 / sum_t ref^2.

    obs, ref: (n_channels, n_t).  Note the measure is a ratio of squares (no root).
    """
    obs = np.asarray(obs, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.sum((obs - ref) ** 2, axis=1)
    den = np.sum(ref ** 2, axis=1)
    return float(np.mean(num / den))


def dense_stiffness(lam, mu, h):
    """Brute-force global K (3N x 3N) by element loops over K_e = h (lam K_lam + mu K_mu).

    Only for tiny grids; the independent plain-loop counterpart of matvec().
    """
    Kl, Km = ovfem_reference()
    nz, ny, nx = lam.shape
    N = (nx + 1) * (ny + 1) * (nz + 1)
    K = np.zeros((3 * N, 3 * N))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                Ke = h * (lam[k, j, i] * Kl + mu[k, j, i] * Km)
                dofs = []
                for alpha in range(8):
                    di, dj, dk = alpha & 1, (alpha >> 1) & 1, (alpha >> 2) & 1
                    node = (i + di) + (nx + 1) * ((j + dj) + (ny + 1) * (k + dk))
                    dofs += [3 * node, 3 * node + 1, 3 * node + 2]
                for a, p in enumerate(dofs):
                    for b, q in enumerate(dofs):
                        K[p, q] += Ke[a, b]
    return K


def matvec_at_nodes(u, lam, mu, h, nodes, solid=None):
    """(K u) at the listed nodes only: each from its (up to 8) touching elements.

    u is the full nodal array (nz+1, ny+1, nx+1, 3); nodes are (k, j, i) triples;
    elements with solid == 0 (removed voxels) contribute nothing, as in Model.
    Used to check full-size results on a sample of outputs.
    """
    Kl, Km = ovfem_reference()
    nz, ny, nx = lam.shape
    out = np.zeros((len(nodes), 3))
    for r, (k, j, i) in enumerate(nodes):
        for alpha in range(8):  # the node is corner alpha of element (i-di, j-dj, k-dk)
            di, dj, dk = alpha & 1, (alpha >> 1) & 1, (alpha >> 2) & 1
            ei, ej, ek = i - di, j - dj, k - dk
            if not (0 <= ei < nx and 0 <= ej < ny and 0 <= ek < nz):
                continue
            if solid is not None and not solid[ek, ej, ei]:
                continue
            ue = np.concatenate([u[ek + ((b >> 2) & 1), ej + ((b >> 1) & 1), ei + (b & 1)] for b in range(8)])
            ye = h * (lam[ek, ej, ei] * (Kl @ ue) + mu[ek, ej, ei] * (Km @ ue))
            out[r] += ye[3 * alpha:3 * alpha + 3]
    return out
