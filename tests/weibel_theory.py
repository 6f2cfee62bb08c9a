"""The Weibel (current-filamentation) instability of two cold electron beams
counter-streaming along z over a neutralising static background (Sec.
5.1.1): its linear theory for a wavevector k along x, across the beams, and
a seeded setup on a periodic 2D x-y box a few cells wide in y.

Linear theory (cold relativistic fluids, beams of density n_b/2 with
four-velocities +-u_b along z, wp^2 = 4 pi n_b q^2 / m, c = 1): for
perturbations exp(i(k x - w t)) the components E_z, B_y decouple from E_x
(the beams' contributions to J_x cancel).  Each beam's momentum along z
responds to E_z with the longitudinal mass gamma^3 m, its velocity along x
to the magnetic force -v_s B_y with the transverse mass gamma m, and the
density bunching (continuity) carries a current v_s dn_s along z; summing
the beams,

    J_z = (i q^2 n_b / (m w)) E_z [1/gamma^3 + k^2 v^2 / (gamma w^2)],

and the transverse wave equation (w^2 - k^2) E_z = -4 pi i w J_z gives

    w^4 - w^2 (k^2 + wp^2/gamma^3) - wp^2 k^2 v^2 / gamma = 0,

whose root w^2 = -Gamma^2 < 0 is the growing mode; for k -> infinity
Gamma -> v wp / sqrt(gamma), the maximum growth rate the paper quotes."""
import numpy as np


def filamentation_growth(k, wp, ub):
    """Growth rate Gamma(k) of the cold symmetric filamentation mode."""
    gb = np.sqrt(1 + ub * ub)
    vb = ub / gb
    a = k * k + wp * wp / gb ** 3
    b = wp * wp * k * k * vb * vb / gb
    g2 = 2 * b / (a + np.sqrt(a * a + 4 * b))  # the positive root, without cancellation
    return float(np.sqrt(g2))


def weibel_max_rate(wp, ub):
    """The paper's maximum growth rate v_b wp / sqrt(gamma_b) (Sec. 5.1.1)."""
    gb = np.sqrt(1 + ub * ub)
    return ub / gb * wp / np.sqrt(gb)


def setup(nx=128, ny=2, ppc=32, wp=0.2, ub=0.5, temp=1e-4, seed=2512, coupling=4 * np.pi):
    """Two beams of electrons (q = -1, m = 1), ppc/2 each per cell, uniform in
    the box, drifting along +-z with four-velocity ub, thermal spread
    sqrt(temp); weights such that wp^2 = coupling * (weight per unit volume
    of all electrons).  Quiet start: the second beam's particles sit on the
    first beam's positions with the opposite four-velocities, so the initial
    current vanishes point by point and the seeded mode stands above the
    noise.  Returns (grid dict, species list)."""
    rng = np.random.default_rng(seed)
    ncell = nx * ny
    N = ncell * ppc // 2
    w = wp * wp / coupling / ppc
    cells = np.repeat(np.arange(ncell), ppc // 2)
    offs = np.concatenate([rng.random((N, 2)), np.zeros((N, 1))], 1)
    cell = np.stack([cells % nx, cells // nx, np.zeros(N, int)], 1).astype(np.int32)
    u = rng.normal(scale=np.sqrt(temp), size=(N, 3))
    u[:, 2] += ub
    species = []
    for sgn in (+1.0, -1.0):
        species.append(dict(q=-1.0, m=1.0, cell=cell.copy(), offs=offs.copy(), u=sgn * u,
                            w=np.full(N, w), phi=None, alive=np.ones(N, np.int32)))
    grid = dict(n=(nx, ny, 1), lo=(0.0, 0.0, 0.0), hi=(float(nx), float(ny), 1.0))
    return grid, species


def seed_by(nx, ny, mode, amp, pad=0):
    """Fields [6][1][ny + 2 pad][nx + 2 pad] with B_y (component B2, at
    x = i + 1/2) = amp sin(2 pi mode x / nx) and every other component zero
    (pad: ghost cells included on each side)."""
    x = np.arange(nx + 2 * pad) - pad + 0.5
    EB = np.zeros((6, 1, ny + 2 * pad, nx + 2 * pad))
    EB[4] = amp * np.sin(2 * np.pi * mode * x / nx)
    return EB


def fixed_window_rate(t, log_power, t0=5.0, t1=11.0):
    """Growth rate of the amplitude, half the slope of ln power against t over
    [t0, t1] (after the seed's transients, well before saturation)."""
    t = np.asarray(t)
    sel = (t >= t0) & (t <= t1)
    return np.polyfit(t[sel], np.asarray(log_power)[sel], 1)[0] / 2
