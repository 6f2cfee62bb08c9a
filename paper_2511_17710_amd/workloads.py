"""Seeded synthetic inputs for the particle step (host numpy, FP64).

This module only *draws* inputs: particle positions, four-velocities, weights
and analytic field values in the orthonormal (tetrad) basis at the physical
positions of the Yee points.  It holds none of the step's arithmetic
(interpolation, push, move, deposit, sort, basis conversion of the fields);
both the HIP library and the FP64 reference receive the identical arrays it
returns.  Placing an analytic field at a Yee point needs that point's
physical position, so the grid maps of Sec. 2.4 (r(x^1), theta(x^2)) and the
volume element used for load weights (Sec. 2.1) are written out here as input
geometry.

Workloads (all seeded by numpy SeedSequence(17710 + index)):
  cart2d_64      2D Cartesian 64^2 periodic, e-/e+ 8 ppc each, Maxwell-Juttner
                 theta=0.1, Bz=1 plus U[-0.1,0.1] E at each Yee point, 10 steps
  cart3d_128     3D Cartesian 128^3 periodic, 16 ppc per species, Maxwell-Juttner
                 theta=1 boosted to beta=0.3 along x, B0=1 z plus 32 random plane
                 waves of amplitude 0.05, 100 steps, sort every 5
  qsph_1024x512  2D quasi-spherical (r0=0, vartheta=0: log r), r in [1,20], cold
                 pair plasma 10 ppc, n ~ r^-2, dipole + corotation E (Omega=0.1)
  sph_1024x512   same on the uniform-r spherical metric
  qsph_2048x1024 2D quasi-spherical vartheta=0.3, r in [1,50], 16 ppc,
                 Maxwell-Juttner theta=0.5, uniform n, dipole + corotation
  cart3d_64_adj  3D Cartesian 64^3, 8 ppc, as cart3d_128 with L=64; adjoint
                 loss weights W ~ U[-1,1] on every active edge; K=64, m=8
  cart3d_16_fd   16^3 subcase of cart3d_64_adj for finite differences
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

NG = 2
PI = np.pi
# Yee offsets of (E1,E2,E3,B1,B2,B3) in code units (App. A)
STAGGER = np.array([[0.5, 0, 0], [0, 0.5, 0], [0, 0, 0.5],
                    [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])


@dataclass
class Workload:
    name: str
    geom: str                 # "cart" | "sph" | "qsph"
    dim: int
    n: tuple
    lo: tuple
    hi: tuple
    r0: float = 0.0
    vartheta: float = 0.0
    periodic: tuple = (1, 1, 1)
    rho0: float = 1.0
    cfl: float = 0.45
    steps: int = 10
    sort_every: int = 20
    species: List[dict] = field(default_factory=list)
    fields_tetrad: Optional[np.ndarray] = None   # tetrad basis
    fields_includes_ghosts: int = 0              # 0: active region only (periodic)
    W: Optional[np.ndarray] = None               # adjoint loss weights on J (padded)
    K: int = 0
    ckpt_every: int = 0
    seed: int = 0

    @property
    def nparticles(self):
        return int(sum(s["cell"].shape[0] for s in self.species))

    def padded_shape(self):
        d = [self.n[i] + 2 * NG if i < self.dim else 1 for i in range(3)]
        return (d[2], d[1], d[0])


# ------------------------------------------------------------------ samplers
def maxwell_juttner(rng, n, theta, drift_beta=0.0, chunk=1 << 22):
    """Four-velocities from the Maxwell-Juttner distribution of temperature
    theta (m c^2 units), optionally boosted along +x by drift_beta.

    Rest frame: exact rejection sampling of the kinetic energy e = gamma - 1,
    target density (1+e) sqrt(e(e+2)) exp(-e/theta), proposal Gamma(3/2, theta')
    with theta' > theta; the ratio (1+e) sqrt(e+2) exp(-a e), a = 1/theta - 1/theta',
    is maximised in closed form.  Drift: Zenitani (2015) flipping method.
    """
    out = np.empty((n, 3))
    if n == 0:
        return out
    # choose theta' among a few candidates by acceptance rate (numerical integral)
    ee = np.linspace(0, 60 * theta + 60, 400001)[1:]
    fint = np.trapezoid((1 + ee) * np.sqrt(ee * (ee + 2)) * np.exp(-ee / theta), ee)
    best = None
    for fac in (1.02, 1.05, 1.1, 1.2, 1.35, 1.5, 2.0, 3.0):
        tp = theta * fac
        a = 1.0 / theta - 1.0 / tp
        A, Bq, Cq = 2 * a, 6 * a - 3, 4 * a - 5
        disc = Bq * Bq - 4 * A * Cq
        es = max(0.0, (-Bq + np.sqrt(max(disc, 0.0))) / (2 * A))
        lr = np.log1p(es) + 0.5 * np.log(es + 2) - a * es
        acc = fint / (np.exp(lr) * 0.5 * np.sqrt(PI) * tp ** 1.5)
        if best is None or acc > best[0]:
            best = (acc, tp, a, lr)
    _, tp, a, lrmax = best
    got = 0
    while got < n:
        m = min(chunk, int((n - got) / max(best[0], 1e-3) * 1.2) + 64)
        e = rng.gamma(1.5, tp, size=m)
        lr = np.log1p(e) + 0.5 * np.log(e + 2) - a * e
        keep = np.log(rng.random(m)) <= lr - lrmax
        e = e[keep][: n - got]
        k = e.shape[0]
        umag = np.sqrt(e * (e + 2))
        cz = rng.uniform(-1.0, 1.0, size=k)
        ph = rng.uniform(0.0, 2 * PI, size=k)
        sz = np.sqrt(1.0 - cz * cz)
        out[got:got + k, 0] = umag * sz * np.cos(ph)
        out[got:got + k, 1] = umag * sz * np.sin(ph)
        out[got:got + k, 2] = umag * cz
        got += k
    if drift_beta != 0.0:
        g = np.sqrt(1.0 + np.sum(out * out, axis=1))
        flip = -drift_beta * out[:, 0] / g > rng.random(n)
        out[flip, 0] = -out[flip, 0]
        G = 1.0 / np.sqrt(1.0 - drift_beta ** 2)
        out[:, 0] = G * (out[:, 0] + drift_beta * g)
    return out


def _round_fixed32_offsets(o):
    """Offsets as stored by the FP32 library build: nearest multiple of 2^-32,
    kept below 1."""
    q = np.rint(o * 2.0 ** 32)
    q = np.clip(q, 0.0, 2.0 ** 32 - 1.0)
    return q * 2.0 ** -32


# ------------------------------------------------------------------ geometry of inputs
def _r_of(wl, x1):
    if wl.geom == "sph":
        return wl.lo[0] + x1 * (wl.hi[0] - wl.lo[0]) / wl.n[0]
    Rmin = np.log(wl.lo[0] - wl.r0)
    dR = (np.log(wl.hi[0] - wl.r0) - Rmin) / wl.n[0]
    return wl.r0 + np.exp(Rmin + x1 * dR)


def _theta_of(wl, x2):
    T = x2 * PI / wl.n[1]
    if wl.geom == "sph":
        return T
    v = wl.vartheta
    return T + 2 * v * T * (1 - 2 * T / PI) * (1 - T / PI)


def _volume_element(wl, x1, x2):
    """sqrt(det h) at code coordinates (Sec. 2.4 metric list), for load weights."""
    r = _r_of(wl, x1)
    th = _theta_of(wl, x2)
    if wl.geom == "sph":
        dr = (wl.hi[0] - wl.lo[0]) / wl.n[0]
        h1 = dr
        h2 = r * PI / wl.n[1]
    else:
        Rmin = np.log(wl.lo[0] - wl.r0)
        dR = (np.log(wl.hi[0] - wl.r0) - Rmin) / wl.n[0]
        dT = PI / wl.n[1]
        T = x2 * dT
        v = wl.vartheta
        h1 = dR * np.exp(Rmin + x1 * dR)
        h2 = dT * (1 + 2 * v + 12 * v * (T / PI) * (T / PI - 1)) * r
    return h1 * h2 * r * np.sin(th)


# ------------------------------------------------------------------ particles
def _load_uniform(rng, wl, ppc, dims):
    """Exactly ppc particles per active cell, offsets U[0,1)^D, cell-major order."""
    ncell = int(np.prod(dims))
    cid = np.repeat(np.arange(ncell, dtype=np.int64), ppc)
    cell = np.zeros((cid.shape[0], 3), dtype=np.int32)
    rem = cid.copy()
    for d, nd in enumerate(dims):
        cell[:, d] = rem % nd
        rem //= nd
    offs = np.zeros((cid.shape[0], 3))
    offs[:, : len(dims)] = rng.random((cid.shape[0], len(dims)))
    return cell, offs


def _pair_species(cell, offs, u_e, u_p, w, phi):
    sp = []
    for q, u in ((-1.0, u_e), (1.0, u_p)):
        sp.append(dict(q=q, m=1.0, cell=cell.copy(), offs=offs.copy(), u=u, w=w.copy(),
                       phi=None if phi is None else phi.copy(),
                       alive=np.ones(cell.shape[0], dtype=np.int32)))
    return sp


# ------------------------------------------------------------------ fields
def _yee_phys_cart(wl, c, shape_active):
    """Physical coordinates of component c's Yee points over the active region."""
    n3, n2, n1 = shape_active
    d = [(wl.hi[i] - wl.lo[i]) / wl.n[i] if i < wl.dim else 1.0 for i in range(3)]
    xs = wl.lo[0] + (np.arange(n1) + STAGGER[c, 0]) * d[0]
    ys = wl.lo[1] + (np.arange(n2) + STAGGER[c, 1]) * d[1]
    zs = (wl.lo[2] + (np.arange(n3) + STAGGER[c, 2]) * d[2]) if wl.dim == 3 else np.zeros(1)
    return xs, ys, zs


def _plane_waves(rng, wl, nwaves, amp, B0):
    """B0 z_hat + sum of nwaves plane waves, E_m = amp e_m cos(k.x+psi),
    B_m = amp (k_hat x e_m) cos(k.x+psi), k = 2 pi n_m / L, n_m in {-4..4}^3 minus 0."""
    L = np.array([wl.hi[i] - wl.lo[i] for i in range(3)])
    nvec = []
    while len(nvec) < nwaves:
        v = rng.integers(-4, 5, size=3)
        if wl.dim == 2:
            v[2] = 0
        if np.any(v != 0):
            nvec.append(v)
    nvec = np.array(nvec, dtype=np.float64)
    k = 2 * PI * nvec / L
    khat = k / np.linalg.norm(k, axis=1, keepdims=True)
    e = rng.normal(size=(nwaves, 3))
    e -= np.sum(e * khat, axis=1, keepdims=True) * khat
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    bdir = np.cross(khat, e)
    psi = rng.uniform(0, 2 * PI, size=nwaves)
    shp = (wl.n[2] if wl.dim == 3 else 1, wl.n[1], wl.n[0])
    out = np.zeros((6,) + shp)
    for c in range(6):
        xs, ys, zs = _yee_phys_cart(wl, c, shp)
        amp_c = amp * (e[:, c] if c < 3 else bdir[:, c - 3])
        X = np.exp(1j * np.outer(k[:, 0], xs))            # (m, n1)
        Y = np.exp(1j * np.outer(k[:, 1], ys))            # (m, n2)
        Z = np.exp(1j * np.outer(k[:, 2], zs))            # (m, n3)
        A = amp_c * np.exp(1j * psi)
        ZY = (A[:, None, None] * Z[:, :, None] * Y[:, None, :]).reshape(nwaves, -1)  # (m, n3*n2)
        out[c] = np.real(ZY.T @ X).reshape(shp)
    out[5] += B0
    return out


def _dipole_corotation(wl, omega):
    """Tetrad-basis dipole B_r = 2 cos(th)/r^3, B_th = sin(th)/r^3 and the
    corotation field E = -(Omega x r) x B, at every padded Yee point."""
    shp = wl.padded_shape()
    out = np.zeros((6,) + shp)
    n2p, n1p = shp[1], shp[2]
    i = np.arange(n1p) - NG
    j = np.arange(n2p) - NG
    for c in range(6):
        r = _r_of(wl, i + STAGGER[c, 0])[None, :]
        th = _theta_of(wl, j + STAGGER[c, 1])[:, None]
        Br = 2 * np.cos(th) / r ** 3
        Bt = np.sin(th) / r ** 3
        if c == 0:
            v = omega * r * np.sin(th) * Bt
        elif c == 1:
            v = -omega * r * np.sin(th) * Br
        elif c == 3:
            v = Br
        elif c == 4:
            v = Bt
        else:
            v = np.zeros_like(r * th)
        out[c, 0] = np.broadcast_to(v, (n2p, n1p))
    return out


# ------------------------------------------------------------------ workloads
def _streams(index, seed):
    ss = np.random.SeedSequence(17710 + index if seed is None else seed)
    return [np.random.default_rng(s) for s in ss.spawn(5)]


def cart2d(n=64, ppc=8, theta=0.1, steps=10, seed=None, index=1, shuffle=False):
    rp, ru, rf, _, _ = _streams(index, seed)
    wl = Workload(name=f"cart2d_{n}", geom="cart", dim=2, n=(n, n, 1), lo=(0.0, 0.0, 0.0),
                  hi=(float(n), float(n), 1.0), steps=steps, sort_every=20, seed=index)
    cell, offs = _load_uniform(rp, wl, ppc, (n, n))
    N = cell.shape[0]
    ue = maxwell_juttner(ru, N, theta)
    up = maxwell_juttner(ru, N, theta)
    wl.species = _pair_species(cell, offs, ue, up, np.ones(N), None)
    f = np.zeros((6, 1, n, n))
    f[0:3] = rf.uniform(-0.1, 0.1, size=(3, 1, n, n))
    f[5] = 1.0
    wl.fields_tetrad = f
    wl.fields_includes_ghosts = 0
    if shuffle:
        _shuffle(rp, wl)
    return wl


def cart3d(n=128, ppc=16, theta=1.0, drift=0.3, steps=100, nwaves=32, amp=0.05, seed=None,
           index=2, name=None, shuffle=False, sort_every=5):
    """3D periodic pair plasma.  The sort cadence of 5 steps keeps every
    1024-particle chunk of a brick within the LDS tiles of the push kernel:
    at CFL 0.45 and theta = 1 the chunk's bounding box grows by about one cell
    per step, and once box plus stencil halo exceeds about 11.8^3 cells its
    outlying particles read the fields and deposit in global memory."""
    rp, ru, rf, rw, rW = _streams(index, seed)
    wl = Workload(name=name or f"cart3d_{n}", geom="cart", dim=3, n=(n, n, n),
                  lo=(0.0, 0.0, 0.0), hi=(float(n),) * 3, steps=steps, sort_every=sort_every,
                  seed=index)
    cell, offs = _load_uniform(rp, wl, ppc, (n, n, n))
    N = cell.shape[0]
    ue = maxwell_juttner(ru, N, theta, drift)
    up = maxwell_juttner(ru, N, theta, drift)
    wl.species = _pair_species(cell, offs, ue, up, np.ones(N), None)
    wl.fields_tetrad = _plane_waves(rw, wl, nwaves, amp, 1.0)
    wl.fields_includes_ghosts = 0
    if shuffle:
        _shuffle(rp, wl)
    return wl


def cart3d_adjoint(n=64, ppc=8, K=64, ckpt=8, seed=None, index=5):
    wl = cart3d(n=n, ppc=ppc, steps=K, seed=seed, index=index, sort_every=4,
                name=("cart3d_64_adj" if n == 64 else f"cart3d_{n}_adj"))
    rW = _streams(index, seed)[4]
    W = np.zeros((3,) + wl.padded_shape())
    W[:, NG:NG + n, NG:NG + n, NG:NG + n] = rW.uniform(-1, 1, size=(3, n, n, n))
    wl.W = W
    wl.K = K
    wl.ckpt_every = ckpt
    return wl


def curvilinear(geom="qsph", n1=1024, n2=512, rmax=20.0, vartheta=0.0, ppc=10, theta=None,
                density_power=2, steps=200, omega=0.1, seed=None, index=3, shuffle=False):
    rp, ru, rf, _, _ = _streams(index, seed)
    tag = f"{geom}_{n1}x{n2}"
    wl = Workload(name=tag, geom=geom, dim=2, n=(n1, n2, 1), lo=(1.0, 0.0, 0.0),
                  hi=(float(rmax), PI, 1.0), r0=0.0, vartheta=vartheta, periodic=(0, 0, 0),
                  steps=steps, sort_every=20, seed=index)
    cell, offs = _load_uniform(rp, wl, ppc, (n1, n2))
    N = cell.shape[0]
    phi = rp.uniform(0, 2 * PI, size=N)
    x1 = cell[:, 0] + offs[:, 0]
    x2 = cell[:, 1] + offs[:, 1]
    V0 = _volume_element(wl, 0.5, 0.5)
    w = _volume_element(wl, x1, x2) / V0
    if density_power:
        w = w * _r_of(wl, x1) ** (-density_power)
    if theta is None:
        ue = np.zeros((N, 3))
        up = np.zeros((N, 3))
    else:
        ue = maxwell_juttner(ru, N, theta)
        up = maxwell_juttner(ru, N, theta)
    wl.species = _pair_species(cell, offs, ue, up, w, phi)
    wl.fields_tetrad = _dipole_corotation(wl, omega)
    wl.fields_includes_ghosts = 1
    if shuffle:
        _shuffle(rp, wl)
    return wl


def _shuffle(rng, wl):
    for s in wl.species:
        p = rng.permutation(s["cell"].shape[0])
        for k in ("cell", "offs", "u", "w", "phi", "alive"):
            if s.get(k) is not None:
                s[k] = s[k][p].copy()


def round_to_f32(wl):
    """Round every particle and field input to what the FP32 library build
    stores (FP32 values; offsets in 32-bit fixed point), as FP64 arrays, so an
    FP32 run and the FP64 reference start from the same state."""
    for s in wl.species:
        s["offs"] = _round_fixed32_offsets(s["offs"])
        s["u"] = s["u"].astype(np.float32).astype(np.float64)
        s["w"] = s["w"].astype(np.float32).astype(np.float64)
        if s.get("phi") is not None:
            ph = s["phi"].astype(np.float32)
            ph = np.where(ph >= np.float32(2 * PI), np.float32(0.0), ph)
            s["phi"] = ph.astype(np.float64)
    wl.fields_tetrad = wl.fields_tetrad.astype(np.float32).astype(np.float64)
    return wl


def by_name(name, **kw):
    """The named workloads at their full sizes (overridable keywords)."""
    if name == "cart2d_64":
        return cart2d(**kw)
    if name == "cart3d_128":
        return cart3d(**kw)
    if name == "qsph_1024x512":
        return curvilinear("qsph", 1024, 512, 20.0, 0.0, ppc=kw.pop("ppc", 10), theta=None,
                           density_power=2, steps=200, index=3, **kw)
    if name == "sph_1024x512":
        return curvilinear("sph", 1024, 512, 20.0, 0.0, ppc=kw.pop("ppc", 10), theta=None,
                           density_power=2, steps=200, index=3, **kw)
    if name == "qsph_2048x1024":
        return curvilinear("qsph", 2048, 1024, 50.0, 0.3, ppc=kw.pop("ppc", 16), theta=0.5,
                           density_power=0, steps=200, index=4, **kw)
    if name == "cart3d_64_adj":
        return cart3d_adjoint(**kw)
    if name == "cart3d_16_fd":
        return cart3d_adjoint(n=16, ppc=8, K=kw.pop("K", 8), ckpt=kw.pop("ckpt", 4), **kw)
    raise KeyError(name)
